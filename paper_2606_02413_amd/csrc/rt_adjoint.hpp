// Reverse mode of the ray tracer: the adjoint of one ray step (central RK4
// step, the two perturbed retraces and the ray-tube area, the chord-sphere
// termination, the free-free segment and its transfer update) and the scatter of
// model-channel adjoints into a per-vertex accumulator.
//
// Paper: "Modeling the Thermal Low-Frequency Radio Sun with Ray Tracing".
//   Ray equations Sec. 2.1, Eq. 4 (normalised form dr/dt = p, dp/dt = -1/2 grad X);
//   perturbation retracing and magnification Eqs. 5-11 (area without the 1/2);
//   transfer with the geometric term Eqs. 2-3, 12; free-free in its
//   Rayleigh-Jeans closed form with the Dulk (1985) Coulomb logarithm.
//
// The derivative taken is that of the discrete forward computed by ray_step,
// with every discrete choice held fixed: the cell of each evaluation, edge
// clamps, the reference axis of the basis, the step floor, the number of steps
// and the termination code.  The local arithmetic is FP32 like the forward's
// model evaluations; the adjoint of the ray state and of the transfer
// accumulates in FP64.
//
// Notation: for a forward quantity q, q_b is d loss / d q.  A model evaluation at
// a point returns n_e and g = grad n_e (Cartesian); its adjoint takes (n_b, g_b),
// returns the adjoint of the point's position, and scatters the adjoints of the
// vertex channels (n_e, dn/dxi_0, dn/dxi_1, dn/dxi_2, T) of the cell's 8 corners.
#pragma once

#include "rt_trace.hpp"

namespace rt {

// ---------------------------------------------------------------------------
// Channel adjoints.  A model evaluation's adjoint is first written to a per-lane
// log entry (cell key, cell fractions, one adjoint per channel); after a run of
// evaluations the log is replayed: entries are summed per corner in registers
// and added to the lane's cell accumulator in LDS (channel ch of corner k at
// v[(kGradChannels k + ch) * kWaveLanes]).  When the lane moves to another cell
// the accumulator keeps the corners the two cells share and sends the others to
// the per-vertex FP64 accumulator with atomics.
// ---------------------------------------------------------------------------
struct GradAcc {
  int key;   // packed index of the cell's corner 0, or -1 when empty
  float* v;
};

constexpr int kLogWords = 4 + kGradChannels;  // key, u, v, w, channel adjoints
constexpr int kLogEntries = 7;                // evaluations logged before a replay

// Entry e, word j at lg[(kLogWords e + j) * kWaveLanes]: key, u, v, w, then
// the adjoints of the channels (n_e, three index gradients, T).  A gradient
// entry writes the three gradient channels (and n_e when it has one), a value
// entry n_e and T; the replay reads only those.
__device__ __forceinline__ void log_grad_entry(float* lg, int e, const Loc& L, bool with_n, float c0, float c1,
                                               float c2, float c3) {
  float* p = lg + e * kLogWords * kWaveLanes;
  p[0] = __int_as_float(L.key);
  p[kWaveLanes] = L.u; p[2 * kWaveLanes] = L.v; p[3 * kWaveLanes] = L.w;
  if (with_n) p[4 * kWaveLanes] = c0;
  p[5 * kWaveLanes] = c1; p[6 * kWaveLanes] = c2; p[7 * kWaveLanes] = c3;
}

__device__ __forceinline__ void log_value_entry(float* lg, int e, const Loc& L, float c0, float c4) {
  float* p = lg + e * kLogWords * kWaveLanes;
  p[0] = __int_as_float(L.key);
  p[kWaveLanes] = L.u; p[2 * kWaveLanes] = L.v; p[3 * kWaveLanes] = L.w;
  p[4 * kWaveLanes] = c0; p[8 * kWaveLanes] = c4;
}

// Move the lane's LDS accumulator to cell `key` (-1: empty it).  Corners shared
// with the old cell (a move by one cell along one axis shares four) keep their
// sums; the old cell's other nonzero channel adjoints go to gacc with FP64
// atomics; then s is added.
__device__ __forceinline__ void acc_replace(const DevGeom& g, GradAcc& A, double* gacc, int key,
                                            const float s[8][kGradChannels]) {
  float old[8][kGradChannels];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int ch = 0; ch < kGradChannels; ++ch) old[k][ch] = A.v[(k * kGradChannels + ch) * kWaveLanes];
  const int s1 = g.n2p, s0 = g.n1 * g.n2p;
  // axis bit b and direction of a unit move (0: none)
  int b = 0, dir = 0;
  if (A.key >= 0 && key >= 0) {
    const int D = key - A.key;
    if (D == 1 || D == -1) { b = 1; dir = D; }
    else if (D == s1 || D == -s1) { b = 2; dir = D > 0 ? 1 : -1; }
    else if (D == s0 || D == -s0) { b = 4; dir = D > 0 ? 1 : -1; }
  }
  if (A.key >= 0) {
    // a key always names a cell whose far corner lies inside the packed grid
    const bool inside = (long long)A.key + s0 + s1 + 1 < (long long)g.n0 * s0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      // old corner k survives when the move goes towards its side of the cell
      const bool keep = dir != 0 && (((k & b) != 0) == (dir > 0));
      const int off = ((k & 4) ? s0 : 0) + ((k & 2) ? s1 : 0) + (k & 1);
      double* dst = gacc + size_t(A.key + off) * kGradChannels;
#pragma unroll
      for (int ch = 0; ch < kGradChannels; ++ch)
        if (!keep && inside && old[k][ch] != 0.0f) unsafeAtomicAdd(dst + ch, double(old[k][ch]));
    }
  }
  // new corner k is old corner ko when the two cells share that vertex (the
  // old sums are read back from LDS, which still holds them, by address)
  float nv[8][kGradChannels];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const bool shared = dir != 0 && (((k & b) != 0) == (dir < 0));
    const int ko = dir > 0 ? (k | b) : (k & ~b);
#pragma unroll
    for (int ch = 0; ch < kGradChannels; ++ch)
      nv[k][ch] = s[k][ch] + (shared ? A.v[(ko * kGradChannels + ch) * kWaveLanes] : 0.0f);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int ch = 0; ch < kGradChannels; ++ch) A.v[(k * kGradChannels + ch) * kWaveLanes] = nv[k][ch];
  }
  A.key = key;
}

__device__ __forceinline__ void acc_add(GradAcc& A, const float s[8][kGradChannels]) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int ch = 0; ch < kGradChannels; ++ch) A.v[(k * kGradChannels + ch) * kWaveLanes] += s[k][ch];
}

// Corner sums of one log entry added to s: a value entry (VALUE) carries n_e
// and T, a gradient entry the three gradient channels and n_e when WITH_N.
__device__ __forceinline__ void entry_add(float s[8][kGradChannels], const float* p, const float W[8], bool value,
                                          bool with_n) {
  if (value) {
    const float c0 = p[4 * kWaveLanes], c4 = p[8 * kWaveLanes];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      s[k][0] = fmaf(W[k], c0, s[k][0]);
      s[k][4] = fmaf(W[k], c4, s[k][4]);
    }
  } else {
    const float c1 = p[5 * kWaveLanes], c2 = p[6 * kWaveLanes], c3 = p[7 * kWaveLanes];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      s[k][1] = fmaf(W[k], c1, s[k][1]);
      s[k][2] = fmaf(W[k], c2, s[k][2]);
      s[k][3] = fmaf(W[k], c3, s[k][3]);
    }
    if (with_n) {
      const float c0 = p[4 * kWaveLanes];
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k][0] = fmaf(W[k], c0, s[k][0]);
    }
  }
}

// Replay log entries [0, n): entry 0 is a value entry when VALUE0, the others
// gradient entries, the last one with an n_e channel when N_LAST.  Entries of
// the accumulator's cell are summed in registers (sa), entries of one other
// cell too (sb); after the loop sa is added to the accumulator and a lane that
// met another cell moves its accumulator there.  The moves (and their atomics)
// of all lanes thus happen at one point of the program rather than wherever
// each lane meets a new cell; a third cell within one replay takes the same
// move early.
template <bool VALUE0, bool N_LAST>
__device__ __forceinline__ void log_replay(const DevGeom& g, GradAcc& A, double* gacc, const float* lg, int n) {
  float sa[8][kGradChannels], sb[8][kGradChannels];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int ch = 0; ch < kGradChannels; ++ch) sa[k][ch] = sb[k][ch] = 0.0f;
  int kb = -1;
#pragma unroll 1
  for (int e = 0; e < n; ++e) {
    const float* p = lg + e * kLogWords * kWaveLanes;
    const int key = __float_as_int(p[0]);
    if (key != A.key && key != kb) {
      if (kb >= 0) {
        acc_add(A, sa);
        acc_replace(g, A, gacc, kb, sb);
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
          for (int ch = 0; ch < kGradChannels; ++ch) sa[k][ch] = sb[k][ch] = 0.0f;
      }
      kb = key;
    }
    const bool value = VALUE0 && e == 0;
    const bool with_n = N_LAST && e == n - 1;
    float W[8];
    weights8(p[kWaveLanes], p[2 * kWaveLanes], p[3 * kWaveLanes], W);
    if (key == A.key) entry_add(sa, p, W, value, with_n);
    else entry_add(sb, p, W, value, with_n);
  }
  acc_add(A, sa);
  if (kb >= 0) acc_replace(g, A, gacc, kb, sb);
}

// Flush the accumulator to gacc (end of the lane's work).
__device__ __forceinline__ void grad_flush(const DevGeom& g, GradAcc& A, double* gacc) {
  float z[8][kGradChannels];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int ch = 0; ch < kGradChannels; ++ch) z[k][ch] = 0.0f;
  acc_replace(g, A, gacc, -1, z);
}

// Trilinear interpolant of 4 channels over one cell and its derivatives along
// the three index axes (corner k = 4 i + 2 j + k').
__device__ __forceinline__ void tri_deriv4(const float4 q[8], float u, float v, float w, float4& val, float4& du,
                                           float4& dv, float4& dw) {
  const float4 w00 = q[1] - q[0], w01 = q[3] - q[2], w10 = q[5] - q[4], w11 = q[7] - q[6];
  const float4 a00 = q[0] + w * w00, a01 = q[2] + w * w01, a10 = q[4] + w * w10, a11 = q[6] + w * w11;
  const float4 v0 = a01 - a00, v1 = a11 - a10;
  const float4 b0 = a00 + v * v0, b1 = a10 + v * v1;
  val = b0 + u * (b1 - b0);
  du = b1 - b0;
  dv = v0 + u * (v1 - v0);
  const float4 c0 = w00 + v * (w01 - w00), c1 = w10 + v * (w11 - w10);
  dw = c0 + u * (c1 - c0);
}

__device__ __forceinline__ void tri_deriv1(const float q[8], float u, float v, float w, float& val, float& du,
                                           float& dv, float& dw) {
  const float w00 = q[1] - q[0], w01 = q[3] - q[2], w10 = q[5] - q[4], w11 = q[7] - q[6];
  const float a00 = q[0] + w * w00, a01 = q[2] + w * w01, a10 = q[4] + w * w10, a11 = q[6] + w * w11;
  const float v0 = a01 - a00, v1 = a11 - a10;
  const float b0 = a00 + v * v0, b1 = a10 + v * v1;
  val = b0 + u * (b1 - b0);
  du = b1 - b0;
  dv = v0 + u * (v1 - v0);
  const float c0 = w00 + v * (w01 - w00), c1 = w10 + v * (w11 - w10);
  dw = c0 + u * (c1 - c0);
}

// Gradients of the continuous index xi_k (k = 0, 1, 2) at an evaluation point of
// a spherical grid: grad xi_0 = r_hat / (r dl), grad xi_1 = theta_hat / (r dth),
// grad xi_2 = phi_hat / (rho dph); plus the unit vectors the Hessians need.
struct SphFrame {
  float rx, ry, rz;   // r_hat
  float tx, ty, tz;   // theta_hat
  float fx, fy;       // phi_hat (z component 0)
  float cx, cy;       // rho_hat (cylindrical radial, z component 0)
  float s0, s1, s2;   // |grad xi_k|
  float rinv, rhoinv, cot;
};

__device__ __forceinline__ void sph_frame(const DevGeom& g, const Loc& L, SphFrame& F) {
  F.rinv = L.rinv;
  F.rx = L.x * L.rinv; F.ry = L.y * L.rinv; F.rz = L.z * L.rinv;
  F.rhoinv = L.rhoinv;
  F.cx = L.axis ? 1.0f : L.x * L.rhoinv;
  F.cy = L.axis ? 0.0f : L.y * L.rhoinv;
  F.fx = -F.cy; F.fy = F.cx;
  const float ct = L.z * L.rinv, st = L.rho * L.rinv;
  F.tx = ct * F.cx; F.ty = ct * F.cy; F.tz = -st;
  F.s0 = g.inv_dl * L.rinv;
  F.s1 = g.inv_dth * L.rinv;
  F.s2 = L.axis ? 0.0f : g.inv_dph * L.rhoinv;
  F.cot = L.axis ? 0.0f : L.z * L.rhoinv;
}

// Adjoint of eval_grad at r_i + d: (n_b, g_b) -> position adjoint q; the
// channel adjoints go to log entry e.
// WITH_N: the evaluation's n_e value has an adjoint (the step rule's stage-1
// value); the other evaluations only feed forces and leave that channel alone.
template <int KIND, bool WITH_N = false>
__device__ __forceinline__ void eval_grad_adj(const DevGeom& g, const RayState& R, CellCache& C, float* lg, int e,
                                              const StepOrigin& O, float dx, float dy, float dz, float gbx, float gby,
                                              float gbz, float nb, float& qx, float& qy, float& qz) {
  Loc L;
  locate<KIND>(g, O, dx, dy, dz, L);
  ensure_cell(g, R.nfg, R.te, C, L.key);
  float4 q[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) q[k] = C.c[k * kWaveLanes];
  float4 val, du, dv, dw;
  tri_deriv4(q, L.u, L.v, L.w, val, du, dv, dw);
  float Gb0, Gb1, Gb2;
  SphFrame F;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    sph_frame(g, L, F);
    Gb0 = F.s0 * (F.rx * gbx + F.ry * gby + F.rz * gbz);
    Gb1 = F.s1 * (F.tx * gbx + F.ty * gby + F.tz * gbz);
    Gb2 = F.s2 * (F.fx * gbx + F.fy * gby);
  } else {
    Gb0 = gbx * g.inv_sp[0];
    Gb1 = gby * g.inv_sp[1];
    Gb2 = gbz * g.inv_sp[2];
  }
  log_grad_entry(lg, e, L, WITH_N, nb, Gb0, Gb1, Gb2);
  // adjoint of the continuous index (zero along an axis held at an edge)
  const float nbe = WITH_N ? nb : 0.0f;
  const float xb0 = L.cl0 ? 0.0f : nbe * du.x + Gb0 * du.y + Gb1 * du.z + Gb2 * du.w;
  const float xb1 = L.cl1 ? 0.0f : nbe * dv.x + Gb0 * dv.y + Gb1 * dv.z + Gb2 * dv.w;
  const float xb2 = L.cl2 ? 0.0f : nbe * dw.x + Gb0 * dw.y + Gb1 * dw.z + Gb2 * dw.w;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    // sum_m xb_m grad xi_m
    const float a0 = xb0 * F.s0, a1 = xb1 * F.s1, a2 = xb2 * F.s2;
    qx = a0 * F.rx + a1 * F.tx + a2 * F.fx;
    qy = a0 * F.ry + a1 * F.ty + a2 * F.fy;
    qz = a0 * F.rz + a1 * F.tz;
    // sum_k G_k H_k g_b, H_k the Hessian of xi_k:
    //   H_0 v = (v - 2 r_hat (r_hat.v)) / (r^2 dl)
    //   H_1 v = (-r_hat (theta_hat.v) - theta_hat (r_hat.v) + cot(theta) phi_hat (phi_hat.v)) / (r^2 dth)
    //   H_2 v = -(rho_hat (phi_hat.v) + phi_hat (rho_hat.v)) / (rho^2 dph)
    const float rg = F.rx * gbx + F.ry * gby + F.rz * gbz;
    const float tg = F.tx * gbx + F.ty * gby + F.tz * gbz;
    const float pg = F.fx * gbx + F.fy * gby;
    const float cg = F.cx * gbx + F.cy * gby;
    const float k0 = val.y * F.s0 * F.rinv;
    const float k1 = val.z * F.s1 * F.rinv;
    const float k2 = val.w * F.s2 * F.rhoinv;
    const float cr = -2.0f * k0 * rg - k1 * tg;    // along r_hat
    const float ctt = -k1 * rg;                    // along theta_hat
    const float cp = k1 * F.cot * pg - k2 * cg;    // along phi_hat
    const float cc = -k2 * pg;                     // along rho_hat
    qx += k0 * gbx + cr * F.rx + ctt * F.tx + cp * F.fx + cc * F.cx;
    qy += k0 * gby + cr * F.ry + ctt * F.ty + cp * F.fy + cc * F.cy;
    qz += k0 * gbz + cr * F.rz + ctt * F.tz;
  } else {
    qx = xb0 * g.inv_sp[0];
    qy = xb1 * g.inv_sp[1];
    qz = xb2 * g.inv_sp[2];
  }
}

// Adjoint of eval_value at r_i + d: (n_b, T_b) -> position adjoint q; the
// channel adjoints go to log entry e.
template <int KIND>
__device__ __forceinline__ void eval_value_adj(const DevGeom& g, const RayState& R, CellCache& C, float* lg, int e,
                                               const StepOrigin& O, float dx, float dy, float dz, float nb, float tb,
                                               float& qx, float& qy, float& qz) {
  Loc L;
  locate<KIND>(g, O, dx, dy, dz, L);
  ensure_cell(g, R.nfg, R.te, C, L.key);
  float qn[8], qt[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    qn[k] = C.c[k * kWaveLanes].x;
    qt[k] = C.t[k * kWaveLanes];
  }
  float vn, dn0, dn1, dn2, vt, dt0, dt1, dt2;
  tri_deriv1(qn, L.u, L.v, L.w, vn, dn0, dn1, dn2);
  tri_deriv1(qt, L.u, L.v, L.w, vt, dt0, dt1, dt2);
  log_value_entry(lg, e, L, nb, tb);
  const float xb0 = L.cl0 ? 0.0f : nb * dn0 + tb * dt0;
  const float xb1 = L.cl1 ? 0.0f : nb * dn1 + tb * dt1;
  const float xb2 = L.cl2 ? 0.0f : nb * dn2 + tb * dt2;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    SphFrame F;
    sph_frame(g, L, F);
    const float a0 = xb0 * F.s0, a1 = xb1 * F.s1, a2 = xb2 * F.s2;
    qx = a0 * F.rx + a1 * F.tx + a2 * F.fx;
    qy = a0 * F.ry + a1 * F.ty + a2 * F.fy;
    qz = a0 * F.rz + a1 * F.tz;
  } else {
    qx = xb0 * g.inv_sp[0];
    qy = xb1 * g.inv_sp[1];
    qz = xb2 * g.inv_sp[2];
  }
}

// d/dx of the segment factor phi(x) = (1 - e^{-x}) / x: its Taylor series
// below |x| = 1/2 (truncation below 3e-9), the closed form above.
__device__ __forceinline__ float segment_dphi(float x) {
  if (fabsf(x) <= 0.5f) {
    // phi'(x) = sum_{k>=1} k (-x)^{k-1} (-1) / (k+1)!
    float s = -9.0f / 3628800.0f;
    s = fmaf(s, x, 8.0f / 362880.0f);
    s = fmaf(s, x, -7.0f / 40320.0f);
    s = fmaf(s, x, 6.0f / 5040.0f);
    s = fmaf(s, x, -5.0f / 720.0f);
    s = fmaf(s, x, 4.0f / 120.0f);
    s = fmaf(s, x, -3.0f / 24.0f);
    s = fmaf(s, x, 2.0f / 6.0f);
    return fmaf(s, x, -0.5f);
  }
  const float e = __builtin_amdgcn_exp2f(-1.44269504089f * x);
  return (e * (1.0f + x) - 1.0f) * rcpf(x * x);
}

// Adjoint of the ray state carried backward along the ray.
struct AdjState {
  double rbx, rby, rbz;   // d loss / d r_i
  double pbx, pby, pbz;   // d loss / d p_i
  double I;               // brightness entering the current segment from behind (back-to-front solution)
};

// One step backward.  R holds the step's start state (r_i, p_i, its grid index,
// the optical depth before the step, n = i) and tp its forward record (field f
// at tp[f * ts]): no model evaluation of the forward step is repeated, and the
// step's derived quantities are recomputed from these with ray_step's
// arithmetic.  S holds the adjoint of the state after the step and the
// brightness behind it, and is replaced by the adjoint of the start state.  `code` is the termination code the forward step returned.
// The evaluation log entries of the central stages (or of the midpoint, on a
// straight line of sight) are left in the log for step_adjoint_flush, so that
// the caller can issue the next step's loads before that replay's atomics.
// The tracing mode is a compile-time choice (kModeLos, kModeNoMag, kModeFull);
// absorption is always on.
template <int KIND, int MODE>
__device__ __forceinline__ void step_adjoint(const AdjointArgs& aa, const RayState& R, const float (&tv)[kTapeFields],
                                             CellCache& C, GradAcc& A, float* lg, int code, double wgt, AdjState& S) {
  static_assert(MODE == kModeLos || MODE == kModeNoMag || MODE == kModeFull, "fixed tracing mode");
  const TraceArgs& a = aa.t;
  const DevGeom& g = a.g;
  double* gacc = aa.gacc;
  constexpr bool refr = MODE != kModeLos;
  constexpr bool mag = MODE == kModeFull;

  // ---------------- forward values: the step's record plus the arithmetic of ray_step ----------------
  StepOrigin O;
  make_origin<KIND>(R, O);
  const float pxf = float(R.px), pyf = float(R.py), pzf = float(R.pz);
  float h, hh = 0.f, hq = 0.f;
  double hd;
  double drx, dry, drz;
  float d2x = 0.f, d2y = 0.f, d2z = 0.f, d3x = 0.f, d3y = 0.f, d3z = 0.f;
  float F1x = 0.f, F1y = 0.f, F1z = 0.f, F2x = 0.f, F2y = 0.f, F2z = 0.f;
  float sx = 0.f, sy = 0.f, sz = 0.f;
  float ni = 0.f;
  bool floored = true;
  if constexpr (refr) {
    ni = tv[kTapeNi];
    floored = !(ni > a.n_floor);
    hd = floored ? a.ds_max_d * rcp64(a.n_floor_d) : a.ds_max_d * rcp64(double(ni));
    h = float(hd);
    hh = 0.5f * h;
    hq = hh * hh;
    F1x = tv[kTapeF1]; F1y = tv[kTapeF1 + 1]; F1z = tv[kTapeF1 + 2];
    F2x = tv[kTapeF2]; F2y = tv[kTapeF2 + 1]; F2z = tv[kTapeF2 + 2];
    sx = tv[kTapeS]; sy = tv[kTapeS + 1]; sz = tv[kTapeS + 2];
    d2x = hh * pxf; d2y = hh * pyf; d2z = hh * pzf;
    d3x = hh * (pxf + hh * F1x); d3y = hh * (pyf + hh * F1y); d3z = hh * (pzf + hh * F1z);
    const double c6 = R.cfd * hd * (1.0 / 6.0);
    drx = hd * R.px + hd * c6 * double(sx);
    dry = hd * R.py + hd * c6 * double(sy);
    drz = hd * R.pz + hd * c6 * double(sz);
  } else {
    h = a.ds_max;
    hd = a.ds_max_d;
    drx = hd * R.px; dry = hd * R.py; drz = hd * R.pz;
  }

  // chord, basis and the perturbed retraces
  const double ds2 = drx * drx + dry * dry + drz * drz;
  const double inv_ds = rsqrt64(ds2);
  const double ds = ds2 * inv_ds;
  double ux = 0, uy = 0, uz = 0;                  // chord direction t
  double e1x = 0, e1y = 0, e1z = 0, e2x = 0, e2y = 0, e2z = 0, ci = 0, eps = 0;
  double s1x = 0, s1y = 0, s1z = 0, s2x = 0, s2y = 0, s2z = 0, det = 1;
  bool ybr = false;
  float lnM = 0.0f;
  const float hh6 = h * h * (1.0f / 6.0f);
  if constexpr (mag) {
    ux = drx * inv_ds; uy = dry * inv_ds; uz = drz * inv_ds;
    double c1x, c1y, c1z;
    ybr = fabs(uz) > 0.9;
    if (ybr) { c1x = uz; c1y = 0.0; c1z = -ux; }
    else { c1x = -uy; c1y = ux; c1z = 0.0; }
    ci = rsqrt64(c1x * c1x + c1y * c1y + c1z * c1z);
    e1x = c1x * ci; e1y = c1y * ci; e1z = c1z * ci;
    e2x = uy * e1z - uz * e1y; e2y = uz * e1x - ux * e1z; e2z = ux * e1y - uy * e1x;
    eps = double(a.eta) * ds;
    // s_j = eps e_j + h^2/6 a_j, a_j the force-difference sums of the record
    s1x = eps * e1x + double(hh6 * tv[kTapeA]);
    s1y = eps * e1y + double(hh6 * tv[kTapeA + 1]);
    s1z = eps * e1z + double(hh6 * tv[kTapeA + 2]);
    s2x = eps * e2x + double(hh6 * tv[kTapeA + 3]);
    s2y = eps * e2y + double(hh6 * tv[kTapeA + 4]);
    s2z = eps * e2z + double(hh6 * tv[kTapeA + 5]);
    det = (s1y * s2z - s1z * s2y) * ux + (s1z * s2x - s1x * s2z) * uy + (s1x * s2y - s1y * s2x) * uz;
    const double mm1 = fabs(det) * rcp64(eps * eps) - 1.0;
    lnM = fast_log1pf(float(mm1));
  }

  // termination and the segment at the chord midpoint
  double lam = 1.0;
  if (code == kHit) lam = crossing<double>(R.rx, R.ry, R.rz, drx, dry, drz, g.r_in, false);
  else if (code == kExit) lam = crossing<double>(R.rx, R.ry, R.rz, drx, dry, drz, g.r_max, true);
  const float hl = 0.5f * float(lam);
  const float mdx = hl * float(drx), mdy = hl * float(dry), mdz = hl * float(drz);
  const float ne_m = tv[kTapeNeM], te_m = tv[kTapeTeM];
  float kn, lnl, cl;
  double dtau;
  {
    const float lt = __builtin_amdgcn_logf(te_m) * 0.69314718056f;
    cl = (te_m >= 2.0e5f) ? 1.0f : 1.5f;
    lnl = (te_m >= 2.0e5f) ? 24.5f + lt - R.lnf : 18.2f + 1.5f * lt - R.lnf;
    kn = kFFCoefF * ne_m * ne_m * lnl * rcpf(R.f2 * te_m * sqrt_fast(te_m));
    dtau = double(kn) * (kRsunCm * lam * hd);
  }
  const double xs = dtau - lam * double(lnM);

  // ---------------- reverse ----------------
  // transfer: T_b = sum_k P_k b_k + P_N T_bc, b_k = T dtau phi(x), P_{k+1} = P_k e^{-x}
  const double P = double(__builtin_amdgcn_exp2f(-1.44269504089f * float(R.lam_tot)));
  const float xf = float(xs);
  const double ex = double(__builtin_amdgcn_exp2f(-1.44269504089f * xf));
  const double phi = double(segment_phi(xf));
  const double dphi = double(segment_dphi(xf));
  const double Pw = wgt * P;
  const double Inext = S.I;
  const double x_b = Pw * (double(te_m) * dtau * dphi - ex * Inext);
  const double dtau_b = Pw * double(te_m) * phi + x_b;
  double te_b = Pw * dtau * phi;
  S.I = ex * Inext + double(te_m) * dtau * phi;

  double lam_b = -double(lnM) * x_b;   // gamma = -lam ln M
  const double lnM_b = -lam * x_b;
  double hd_b = 0.0;
  float ne_m_b;
  {
    const double kn_b = dtau_b * (kRsunCm * lam * hd);
    lam_b += dtau_b * double(kn) * kRsunCm * hd;
    hd_b += dtau_b * double(kn) * kRsunCm * lam;
    // kappa*n = C n_e^2 lnL / (f^2 T^1.5), lnL = c + cl ln T - ln f
    ne_m_b = float(kn_b) * (2.0f * kFFCoefF * ne_m * lnl * rcpf(R.f2 * te_m * sqrt_fast(te_m)));
    te_b += kn_b * double(kn) * rcp64(double(te_m)) * (double(cl) * rcp64(double(lnl)) - 1.5);
  }
  double rbx = 0.0, rby = 0.0, rbz = 0.0;      // this step's contributions to d loss / d r_i
  double drbx = 0.0, drby = 0.0, drbz = 0.0;   // d loss / d (chord)
  {
    float qx, qy, qz;
    eval_value_adj<KIND>(g, R, C, lg, 0, O, mdx, mdy, mdz, ne_m_b, float(te_b), qx, qy, qz);
    rbx += qx; rby += qy; rbz += qz;
    drbx += 0.5 * lam * qx; drby += 0.5 * lam * qy; drbz += 0.5 * lam * qz;
    lam_b += 0.5 * (double(qx) * drx + double(qy) * dry + double(qz) * drz);
  }
  // chord-sphere root: |r + lam dr|^2 = R^2
  if ((code == kHit || code == kExit) && lam > 0.0 && lam < 1.0) {
    const double px = R.rx + lam * drx, py = R.ry + lam * dry, pz = R.rz + lam * drz;
    const double den = px * drx + py * dry + pz * drz;
    if (den != 0.0) {
      const double c = -lam_b * rcp64(den);
      rbx += c * px; rby += c * py; rbz += c * pz;
      drbx += c * lam * px; drby += c * lam * py; drbz += c * lam * pz;
    }
  }

  // central-stage gradient adjoints collected from the perturbed retraces
  float g1bx = 0.f, g1by = 0.f, g1bz = 0.f, g2bx = 0.f, g2by = 0.f, g2bz = 0.f, g3bx = 0.f, g3by = 0.f, g3bz = 0.f;
  float d2bx = 0.f, d2by = 0.f, d2bz = 0.f, d3bx = 0.f, d3by = 0.f, d3bz = 0.f;
  double hq_b = 0.0;
  if constexpr (mag) {
    // ln M = ln|det| - 2 ln eps, det = (s1 x s2) . t
    const double det_b = lnM_b * rcp64(det);
    double eps_b = -2.0 * lnM_b * rcp64(eps);
    const double sb1x = det_b * (s2y * uz - s2z * uy), sb1y = det_b * (s2z * ux - s2x * uz),
                 sb1z = det_b * (s2x * uy - s2y * ux);
    const double sb2x = det_b * (uy * s1z - uz * s1y), sb2y = det_b * (uz * s1x - ux * s1z),
                 sb2z = det_b * (ux * s1y - uy * s1x);
    double tbx = det_b * (s1y * s2z - s1z * s2y), tby = det_b * (s1z * s2x - s1x * s2z),
           tbz = det_b * (s1x * s2y - s1y * s2x);
    double e1bx = 0, e1by = 0, e1bz = 0, e2bx = 0, e2by = 0, e2bz = 0;
#pragma unroll 1
    for (int jj = 0; jj < 2; ++jj) {
      const double ex_ = jj ? e2x : e1x, ey_ = jj ? e2y : e1y, ez_ = jj ? e2z : e1z;
      const double sbx = jj ? sb2x : sb1x, sby = jj ? sb2y : sb1y, sbz = jj ? sb2z : sb1z;
      const float ajx = jj ? tv[kTapeA + 3] : tv[kTapeA], ajy = jj ? tv[kTapeA + 4] : tv[kTapeA + 1],
                  ajz = jj ? tv[kTapeA + 5] : tv[kTapeA + 2];
      const float qjx = jj ? tv[kTapeQ + 3] : tv[kTapeQ], qjy = jj ? tv[kTapeQ + 4] : tv[kTapeQ + 1],
                  qjz = jj ? tv[kTapeQ + 5] : tv[kTapeQ + 2];
      const float fx = float(eps * ex_), fy = float(eps * ey_), fz = float(eps * ez_);
      // s_j = eps e_j + h^2/6 a_j
      eps_b += sbx * ex_ + sby * ey_ + sbz * ez_;
      double ebx = eps * sbx, eby = eps * sby, ebz = eps * sbz;
      const float abx_ = hh6 * float(sbx), aby_ = hh6 * float(sby), abz_ = hh6 * float(sbz);
      hd_b += (double(h) / 3.0) * (double(ajx) * sbx + double(ajy) * sby + double(ajz) * sbz);
      // third stage of the perturbed ray at d3 + d0 + hq q1
      float p3x, p3y, p3z;
      eval_grad_adj<KIND>(g, R, C, lg, 1 + 3 * jj, O, d3x + fx + hq * qjx, d3y + fy + hq * qjy, d3z + fz + hq * qjz,
                          R.cf * abx_, R.cf * aby_, R.cf * abz_, 0.0f, p3x, p3y, p3z);
      rbx += p3x; rby += p3y; rbz += p3z;
      d3bx += p3x; d3by += p3y; d3bz += p3z;
      float d0bx = p3x, d0by = p3y, d0bz = p3z;
      hq_b += double(p3x) * qjx + double(p3y) * qjy + double(p3z) * qjz;
      const float qtx = abx_ + hq * p3x, qty = aby_ + hq * p3y, qtz = abz_ + hq * p3z;  // adjoint of q1
      g3bx -= R.cf * abx_; g3by -= R.cf * aby_; g3bz -= R.cf * abz_;
      // second stage at d2 + d0
      float p2x, p2y, p2z;
      eval_grad_adj<KIND>(g, R, C, lg, 2 + 3 * jj, O, d2x + fx, d2y + fy, d2z + fz, R.cf * abx_, R.cf * aby_,
                          R.cf * abz_, 0.0f, p2x, p2y, p2z);
      rbx += p2x; rby += p2y; rbz += p2z;
      d2bx += p2x; d2by += p2y; d2bz += p2z;
      d0bx += p2x; d0by += p2y; d0bz += p2z;
      g2bx -= R.cf * abx_; g2by -= R.cf * aby_; g2bz -= R.cf * abz_;
      // first stage at d0: q1 = cf G(P1) - F1
      float p1x, p1y, p1z;
      eval_grad_adj<KIND>(g, R, C, lg, 3 + 3 * jj, O, fx, fy, fz, R.cf * qtx, R.cf * qty, R.cf * qtz, 0.0f, p1x, p1y,
                          p1z);
      rbx += p1x; rby += p1y; rbz += p1z;
      d0bx += p1x; d0by += p1y; d0bz += p1z;
      g1bx -= R.cf * qtx; g1by -= R.cf * qty; g1bz -= R.cf * qtz;
      // d0 = eps e_j
      eps_b += double(d0bx) * ex_ + double(d0by) * ey_ + double(d0bz) * ez_;
      ebx += eps * d0bx; eby += eps * d0by; ebz += eps * d0bz;
      if (jj == 0) { e1bx += ebx; e1by += eby; e1bz += ebz; }
      else { e2bx += ebx; e2by += eby; e2bz += ebz; }
    }
    log_replay<true, false>(g, A, gacc, lg, 7);
    // e2 = t x e1
    tbx += e1y * e2bz - e1z * e2by; tby += e1z * e2bx - e1x * e2bz; tbz += e1x * e2by - e1y * e2bx;
    e1bx += e2by * uz - e2bz * uy; e1by += e2bz * ux - e2bx * uz; e1bz += e2bx * uy - e2by * ux;
    // e1 = c1 / |c1|
    const double ed = e1x * e1bx + e1y * e1by + e1z * e1bz;
    const double c1bx = ci * (e1bx - e1x * ed), c1by = ci * (e1by - e1y * ed), c1bz = ci * (e1bz - e1z * ed);
    if (ybr) { tbz += c1bx; tbx -= c1bz; }   // c1 = (t_z, 0, -t_x)
    else { tby -= c1bx; tbx += c1by; }       // c1 = (-t_y, t_x, 0)
    // eps = eta ds; t = dr / ds; ds = |dr|
    const double ds_b = double(a.eta) * eps_b;
    const double tt = ux * tbx + uy * tby + uz * tbz;
    drbx += (tbx - ux * tt) * inv_ds + ds_b * ux;
    drby += (tby - uy * tt) * inv_ds + ds_b * uy;
    drbz += (tbz - uz * tt) * inv_ds + ds_b * uz;
  }

  // central step: r_{i+1} = r_i + dr, p_{i+1} = p_i + dp
  drbx += S.rbx; drby += S.rby; drbz += S.rbz;
  rbx += S.rbx; rby += S.rby; rbz += S.rbz;
  double pbx = S.pbx, pby = S.pby, pbz = S.pbz;
  if constexpr (refr) {
    // log entries of the central stages: after the midpoint value (entry 0) unless
    // the perturbed retraces' replay has already taken it
    const int e0 = mag ? 0 : 1;
    const double dpbx = S.pbx, dpby = S.pby, dpbz = S.pbz;
    // dr = h p + (h^2 / 6) cf s, dp = (h / 6) cf t
    hd_b += drbx * R.px + drby * R.py + drbz * R.pz +
            (hd / 3.0) * R.cfd * (drbx * double(sx) + drby * double(sy) + drbz * double(sz));
    pbx += hd * drbx; pby += hd * drby; pbz += hd * drbz;
    const double ks = hd * hd * (1.0 / 6.0) * R.cfd;
    const float sbx = float(ks * drbx), sby = float(ks * drby), sbz = float(ks * drbz);
    hd_b += (R.cfd / 6.0) * (dpbx * double(tv[kTapeT]) + dpby * double(tv[kTapeT + 1]) +
                             dpbz * double(tv[kTapeT + 2]));
    const double kt = hd * (1.0 / 6.0) * R.cfd;
    const float tbx_ = float(kt * dpbx), tby_ = float(kt * dpby), tbz_ = float(kt * dpbz);
    g1bx += sbx + tbx_; g1by += sby + tby_; g1bz += sbz + tbz_;
    g2bx += sbx + 2.f * tbx_; g2by += sby + 2.f * tby_; g2bz += sbz + 2.f * tbz_;
    g3bx += sbx + 2.f * tbx_; g3by += sby + 2.f * tby_; g3bz += sbz + 2.f * tbz_;
    float qx, qy, qz;
    // fourth stage at d4 = h (p + hh F2) = h p + (h^2 / 2) cf g2
    eval_grad_adj<KIND>(g, R, C, lg, e0, O, h * (pxf + hh * F2x), h * (pyf + hh * F2y), h * (pzf + hh * F2z), tbx_,
                        tby_, tbz_, 0.0f, qx, qy, qz);
    rbx += qx; rby += qy; rbz += qz;
    hd_b += double(qx) * (R.px + hd * double(F2x)) + double(qy) * (R.py + hd * double(F2y)) +
            double(qz) * (R.pz + hd * double(F2z));
    pbx += hd * qx; pby += hd * qy; pbz += hd * qz;
    const float k4 = 0.5f * h * h * R.cf;
    g2bx += k4 * qx; g2by += k4 * qy; g2bz += k4 * qz;
    // third stage at d3 = hh p + hq cf g1
    eval_grad_adj<KIND>(g, R, C, lg, e0 + 1, O, d3x, d3y, d3z, g3bx, g3by, g3bz, 0.0f, qx, qy, qz);
    rbx += qx; rby += qy; rbz += qz;
    d3bx += qx; d3by += qy; d3bz += qz;
    hd_b += double(d3bx) * (0.5 * R.px + 0.5 * hd * double(F1x)) + double(d3by) * (0.5 * R.py + 0.5 * hd * double(F1y)) +
            double(d3bz) * (0.5 * R.pz + 0.5 * hd * double(F1z));
    pbx += 0.5 * hd * d3bx; pby += 0.5 * hd * d3by; pbz += 0.5 * hd * d3bz;
    const float k3 = hq * R.cf;
    g1bx += k3 * d3bx; g1by += k3 * d3by; g1bz += k3 * d3bz;
    // second stage at d2 = hh p
    eval_grad_adj<KIND>(g, R, C, lg, e0 + 2, O, d2x, d2y, d2z, g2bx, g2by, g2bz, 0.0f, qx, qy, qz);
    rbx += qx; rby += qy; rbz += qz;
    d2bx += qx; d2by += qy; d2bz += qz;
    hd_b += 0.5 * (double(d2bx) * R.px + double(d2by) * R.py + double(d2bz) * R.pz);
    pbx += 0.5 * hd * d2bx; pby += 0.5 * hd * d2by; pbz += 0.5 * hd * d2bz;
    // hq = h^2 / 4
    hd_b += hq_b * 0.5 * hd;
    // dt = ds_max / n(r_i), n = sqrt(1 - Xf n_e)
    float ne1_b = 0.0f;
    if (!floored) {
      const double rni = rcp64(double(ni));
      const double n_b = -(hd * rni) * hd_b;
      ne1_b = float(-(0.5 * double(R.xff) * rni) * n_b);
    }
    // first stage at r_i (gradient and the value that set the step)
    eval_grad_adj<KIND, true>(g, R, C, lg, e0 + 3, O, 0.f, 0.f, 0.f, g1bx, g1by, g1bz, ne1_b, qx, qy, qz);
    rbx += qx; rby += qy; rbz += qz;
  } else {
    pbx += hd * drbx; pby += hd * drby; pbz += hd * drbz;
  }
  S.rbx = rbx; S.rby = rby; S.rbz = rbz;
  S.pbx = pbx; S.pby = pby; S.pbz = pbz;
}

// Replay of the log entries step_adjoint leaves: the central stages (after the
// midpoint value when the perturbed retraces' replay has not taken it), or the
// midpoint alone on a straight line of sight.
template <int MODE>
__device__ __forceinline__ void step_adjoint_flush(const DevGeom& g, GradAcc& A, double* gacc, float* lg) {
  if constexpr (MODE == kModeFull) log_replay<false, true>(g, A, gacc, lg, 4);
  else if constexpr (MODE == kModeNoMag) log_replay<true, true>(g, A, gacc, lg, 5);
  else log_replay<true, false>(g, A, gacc, lg, 1);
}

// ---------------------------------------------------------------------------
// Checkpoints and the per-step buffer: [entry][field][slot] FP64.
// ---------------------------------------------------------------------------
// (entries outside [0, limit) are never addressed; the bound is a guard)
__device__ __forceinline__ void state_store(double* buf, int entry, int limit, int n_slots, int slot,
                                            const RayState& R) {
  if ((unsigned)entry >= (unsigned)limit) return;
  double* p = buf + size_t(entry) * kCkptFields * size_t(n_slots) + slot;
  const size_t s = size_t(n_slots);
  p[0] = R.rx; p[s] = R.ry; p[2 * s] = R.rz;
  p[3 * s] = R.px; p[4 * s] = R.py; p[5 * s] = R.pz;
  p[6 * s] = R.b0; p[7 * s] = R.b1; p[8 * s] = R.b2;
  p[9 * s] = R.lam_tot;
}

__device__ __forceinline__ void state_load(const double* buf, int entry, int limit, int n_slots, int slot,
                                           RayState& R) {
  if ((unsigned)entry >= (unsigned)limit) return;
  const double* p = buf + size_t(entry) * kCkptFields * size_t(n_slots) + slot;
  const size_t s = size_t(n_slots);
  R.rx = p[0]; R.ry = p[s]; R.rz = p[2 * s];
  R.px = p[3 * s]; R.py = p[4 * s]; R.pz = p[5 * s];
  R.b0 = p[6 * s]; R.b1 = p[7 * s]; R.b2 = p[8 * s];
  R.lam_tot = p[9 * s];
  R.code = kRunning;
}

// Record of chunk step `entry` (0 <= entry < K, which the chunk loop keeps).
__device__ __forceinline__ float* tape_entry(const AdjointArgs& aa, int entry, int slot) {
  return aa.tape + size_t(entry) * kTapeFields * size_t(aa.n_slots) + slot;
}

// The fields of a step's record that the mode's backward step reads, all
// loaded at once (one memory round trip per step instead of one per use).
template <int MODE>
__device__ __forceinline__ void tape_read(const float* tp, size_t ts, float (&tv)[kTapeFields]) {
#pragma unroll
  for (int f = 0; f < kTapeFields; ++f) {
    const bool used = (f == kTapeNeM || f == kTapeTeM) || (MODE != kModeLos && f < kTapeQ) ||
                      (MODE == kModeFull && f >= kTapeQ && f < kTapeNeM);
    tv[f] = used ? tp[size_t(f) * ts] : 0.0f;
  }
}

__device__ __forceinline__ void state_copy(double* buf, int from, int to, int limit, int n_slots, int slot) {
  if ((unsigned)from >= (unsigned)limit || (unsigned)to >= (unsigned)limit) return;
  const size_t s = size_t(n_slots);
  const double* src = buf + size_t(from) * kCkptFields * s + slot;
  double* dst = buf + size_t(to) * kCkptFields * s + slot;
  for (int f = 0; f < kCkptFields; ++f) dst[f * s] = src[f * s];
}

// Forward pass of one ray for the adjoint: the trace with its state
// checkpointed every kr steps (kr starts at K and doubles, with every other
// checkpoint dropped, whenever the ray outgrows the checkpoint capacity) in the
// ray's own column rid of ckpt.  Adds w T_b to `loss`, writes T_b and the
// ray's record for the sweep: the step count (0 when the ray is not swept:
// a miss, a non-finite step or w = 0), the termination code and checkpoint
// count, and kr.
template <int KIND, int MODE>
__device__ __forceinline__ void adjoint_forward_ray(const AdjointArgs& aa, int img, int pix, int rid, CellCache& C,
                                                    double& loss) {
  const TraceArgs& a = aa.t;
  const int id = img * (a.nu * a.nv) + pix;
  const double wgt = double(aa.weights[id]);
  const size_t nr = size_t(aa.n_rays);
  RayState R;
  if (!init_ray(a, img, pix, R, C)) {
    loss += wgt * a.tb_sky;
    aa.meta[rid] = 0;
    return;
  }
  const int K = aa.K;
  int kr = K, nc = 0, code;
  do {
    if (R.n % kr == 0) {
      if (nc == aa.ckpt_cap) {
        for (int j = 1; j < nc / 2; ++j) state_copy(aa.ckpt, 2 * j, j, aa.ckpt_cap, aa.n_rays, rid);
        nc /= 2;
        kr *= 2;
      }
      state_store(aa.ckpt, nc, aa.ckpt_cap, aa.n_rays, rid, R);
      ++nc;
    }
    code = ray_step<true, KIND, MODE, true>(a, R, C, nullptr, 0);
  } while (code == kRunning);
  finish_ray(a, R);
  const double tbc = (code == kHit) ? a.tb_inner : a.tb_sky;
  const float trans = __builtin_amdgcn_exp2f(-1.44269504089f * float(R.lam_tot));
  loss += wgt * double(float(R.A + double(trans) * tbc));
  aa.meta[rid] = (code == kNonfinite || wgt == 0.0) ? 0 : R.n;
  aa.meta[nr + rid] = code | (nc << 8);
  aa.meta[2 * nr + rid] = kr;
}

// Reverse sweep of one ray, segment by segment from its checkpoints: each chunk
// of at most K steps is recomputed from its checkpoint, writing each step's
// start state and forward record into the lane's slot, and swept backward.
template <int KIND, int MODE>
__device__ __forceinline__ void adjoint_reverse_ray(const AdjointArgs& aa, int img, int pix, int rid, int slot,
                                                    CellCache& C, GradAcc& A, float* lg) {
  const TraceArgs& a = aa.t;
  const size_t nr = size_t(aa.n_rays);
  const int N = aa.meta[rid];
  if (N <= 0) return;
  const int code = aa.meta[nr + rid] & 0xff, nc = aa.meta[nr + rid] >> 8, kr = aa.meta[2 * nr + rid];
  const double wgt = double(aa.weights[img * (a.nu * a.nv) + pix]);
  RayState R;
  if (!init_ray(a, img, pix, R, C)) return;  // (not reached: a swept ray is no miss)
  const int K = aa.K;
  const size_t ts = size_t(aa.n_slots);
  AdjState S;
  S.rbx = S.rby = S.rbz = 0.0;
  S.pbx = S.pby = S.pbz = 0.0;
  S.I = (code == kHit) ? a.tb_inner : a.tb_sky;
  for (int seg = nc - 1; seg >= 0; --seg) {
    const int s0 = seg * kr, s1 = min(N, s0 + kr);
    for (int c1 = s1; c1 > s0; c1 -= K) {
      const int c0 = max(s0, c1 - K);
      state_load(aa.ckpt, seg, aa.ckpt_cap, aa.n_rays, rid, R);
      R.n = s0;
      // steps s0 .. c0-1 are only retraced; steps c0 .. c1-1 are recorded
      while (R.n < c1) {
        float* tp = nullptr;
        if (R.n >= c0) {
          state_store(aa.steps, R.n - c0, aa.K, aa.n_slots, slot, R);
          tp = tape_entry(aa, R.n - c0, slot);
        }
        ray_step<true, KIND, MODE, true>(a, R, C, tp, ts);
      }
      // the next (earlier) step's state and record are loaded before the
      // replay of this step's last log entries issues its atomics
      float tv[kTapeFields];
      state_load(aa.steps, c1 - 1 - c0, aa.K, aa.n_slots, slot, R);
      tape_read<MODE>(tape_entry(aa, c1 - 1 - c0, slot), ts, tv);
      for (int i = c1 - 1; i >= c0; --i) {
        R.n = i;
        step_adjoint<KIND, MODE>(aa, R, tv, C, A, lg, (i == N - 1) ? code : kRunning, wgt, S);
        if (i > c0) {
          state_load(aa.steps, i - 1 - c0, aa.K, aa.n_slots, slot, R);
          tape_read<MODE>(tape_entry(aa, i - 1 - c0, slot), ts, tv);
        }
        step_adjoint_flush<MODE>(a.g, A, aa.gacc, lg);
      }
    }
  }
  // launch: p0 = n(r0) (-o), n(r0) from n_e at the start point (R holds step 0)
  if constexpr (MODE != kModeLos) {
    const float ne0 = a.launch_ne[pix];
    const float n2 = 1.0f - R.xff * ne0;
    if (n2 > 0.f) {
      const float nidx = sqrt_fast(n2);
      const double n_b = -(a.o[0] * S.pbx + a.o[1] * S.pby + a.o[2] * S.pbz);
      const float ne_b = float(-(0.5 * double(R.xff) * rcp64(double(nidx))) * n_b);
      StepOrigin O;
      make_origin<KIND>(R, O);
      float qx, qy, qz;
      eval_value_adj<KIND>(a.g, R, C, lg, 0, O, 0.f, 0.f, 0.f, ne_b, 0.0f, qx, qy, qz);
      log_replay<true, false>(a.g, A, aa.gacc, lg, 1);
    }
  }
}

}  // namespace rt
