// Per-ray device code: model gathers, one RK4 step with step-wise perturbation
// retracing, free-free segment transfer, launch and finish.
//
// Paper: "Modeling the Thermal Low-Frequency Radio Sun with Ray Tracing".
//   Ray equations: Sec. 2.1, Eq. 4, in the normalised form dr/dt = p,
//   dp/dt = -1/2 grad X with X = (8.98e3)^2 n_e / f^2 (|p| = n, ds = n dt).
//   Perturbation retracing and magnification: Eqs. 5-11 (area without the 1/2).
//   Transfer with the geometric term: Eqs. 2-3, 12; one exact exponential
//   update per segment, composited front to back (same products as the
//   back-to-front solution of Sec. 3.2).
//   Free-free: Rayleigh-Jeans closed form with the two-branch Coulomb
//   logarithm of Dulk (1985).
#pragma once

#include "rt_internal.hpp"

namespace rt {

constexpr float kTwoPiF = 6.28318530717958647692f;
constexpr double kRsunCm = 6.957e10;
constexpr float kFFCoefF = 9.78e-3f;

enum : int { kRunning = 0, kExit = 1, kHit = 2, kMiss = 3, kMaxSteps = 4, kNonfinite = 5 };

template <bool MIXED> struct RealOf { using T = double; };
template <> struct RealOf<false> { using T = float; };

// The 8 corners of the last cell a lane touched, kept in LDS: (n_e, index-space
// gradient) and T of corner k = 4 i + 2 j + k' for offsets (i, j, k') along axes
// 0, 1, 2.  Slots are corner-major ([corner][lane]) so that the 64 lanes of a
// wave read consecutive 16-byte words (no bank conflicts).  Each lane only reads
// its own slots, which it wrote itself; LDS operations of a wave complete in order.
constexpr int kWaveLanes = 64;
struct CellCache {
  int key;
  float4* c;  // LDS, corner k at c[k * kWaveLanes]
  float* t;   // LDS, corner k at t[k * kWaveLanes]
};

// Grid coordinates of a step's origin r_i, computed once per step in FP64 from
// the compensated position.  Every evaluation point of the step is r_i + d
// with a small FP32 offset d; its continuous grid index is the origin's FP64
// index plus an FP32 increment from cancellation-free small-offset formulas.
// FP32 alone cannot place a point inside a cell to better than
// ulp(r)/(r dl) ~ 1e-6..5e-6 of a cell, which would perturb every force by
// ~1e-6 and move exit points by ~1e-4 R_sun after a strongly refracted path.
struct StepOrigin {
  float x, y, z;        // r_i rounded to FP32 (for the offset formulas)
  float r2, rho2, rho;  // |r_i|^2, rho_i^2, rho_i
  double b0, b1, b2;    // continuous grid index of r_i
};

template <int KIND>
__device__ __forceinline__ void make_origin(const DevGeom& g, double X, double Y, double Z, StepOrigin& O) {
  O.x = float(X); O.y = float(Y); O.z = float(Z);
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    const double rho2 = X * X + Y * Y;
    const double r2 = rho2 + Z * Z;
    const double rho = sqrt(rho2);
    O.r2 = float(r2); O.rho2 = float(rho2); O.rho = float(rho);
    O.b0 = (0.5 * log(r2) - double(g.ln_rin_d)) * g.inv_dl_d;
    O.b1 = atan2(rho, Z) * g.inv_dth_d - 0.5;
    double ph = (rho2 > 0.0) ? atan2(Y, X) : 0.0;
    if (ph < 0.0) ph += 6.283185307179586476925;
    O.b2 = ph * g.inv_dph_d;
  } else {
    O.r2 = 0.f; O.rho2 = 0.f; O.rho = 0.f;
    O.b0 = (X - double(g.org_d[0])) * g.inv_sp_d[0];
    O.b1 = (Y - double(g.org_d[1])) * g.inv_sp_d[1];
    O.b2 = (Z - double(g.org_d[2])) * g.inv_sp_d[2];
  }
}

struct Loc {
  int key;
  float u, v, w;
  bool clamp0, clamp1, clamp2;
  // spherical chain-rule pieces at the evaluation point
  float rinv, rho, rhoinv, x, y, z;
  bool axis;
};

// Clamp a continuous index to [0, n-1] (NaN -> 0); report whether it was outside.
__device__ __forceinline__ double clamp_index(double xi, int n, bool& clamped) {
  clamped = false;
  if (!(xi >= 0.0)) { clamped = true; return 0.0; }
  const double hi = double(n - 1);
  if (xi > hi) { clamped = true; return hi; }
  return xi;
}

template <int KIND>
__device__ __forceinline__ void locate(const DevGeom& g, const StepOrigin& O, float dx, float dy, float dz, Loc& L) {
  double x0, x1, x2;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    // radius: |q|^2 = |r_i|^2 (1 + c / |r_i|^2), c = 2 r_i.d + |d|^2
    const float rd = O.x * dx + O.y * dy;
    const float c = 2.0f * (rd + O.z * dz) + (dx * dx + dy * dy + dz * dz);
    const float lr = log1pf(c / O.r2);
    x0 = O.b0 + double(0.5f * lr * g.inv_dl);
    // azimuth: angle from (x_i, y_i) to (x_i + dx, y_i + dy)
    const float dphi = atan2f(O.x * dy - O.y * dx, O.rho2 + O.x * dx + O.y * dy);
    x2 = O.b2 + double(dphi * g.inv_dph);
    // colatitude: angle from (z_i, rho_i) to (z_q, rho_q) in the meridional plane
    const float e = 2.0f * rd + (dx * dx + dy * dy);
    const float rho2q = fmaxf(O.rho2 + e, 0.0f);
    const float rhoq = sqrtf(rho2q);
    const float den_r = rhoq + O.rho;
    const float drho = den_r > 0.0f ? e / den_r : 0.0f;
    const float zq = O.z + dz;
    const float dth = atan2f(O.z * drho - O.rho * dz, O.z * zq + O.rho * rhoq);
    x1 = O.b1 + double(dth * g.inv_dth);
    const float r2q = O.r2 + c;
    L.rinv = rsqrtf(r2q);
    L.rho = rhoq;
    L.axis = rhoq < 1e-12f;
    L.rhoinv = L.axis ? 0.0f : 1.0f / rhoq;
    L.x = O.x + dx; L.y = O.y + dy; L.z = zq;
  } else {
    x0 = O.b0 + double(dx * g.inv_sp[0]);
    x1 = O.b1 + double(dy * g.inv_sp[1]);
    x2 = O.b2 + double(dz * g.inv_sp[2]);
  }
  bool c0, c1, c2 = false;
  const double xr = clamp_index(x0, g.n0, c0);
  const double xt = clamp_index(x1, g.n1, c1);
  const int a = min(int(floor(xr)), g.n0 - 2);
  const int b = min(int(floor(xt)), g.n1 - 2);
  int c;
  double xp;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    // periodic phi: wrap into [0, n2)
    xp = x2;
    if (!(xp >= 0.0 && xp < 4.0 * g.n2)) xp = (xp >= -4.0 * g.n2) ? xp + 4.0 * g.n2 : 0.0;  // NaN / far guard
    const double fl = floor(xp);
    c = int(fl);
    c %= g.n2;
    L.w = float(xp - fl);
  } else {
    xp = clamp_index(x2, g.n2, c2);
    c = min(int(floor(xp)), g.n2 - 2);
    L.w = float(xp - double(c));
  }
  L.key = (a * g.n1 + b) * g.n2p + c;
  L.u = float(xr - double(a));
  L.v = float(xt - double(b));
  L.clamp0 = c0; L.clamp1 = c1; L.clamp2 = c2;
}

__device__ __forceinline__ void ensure_cell(const DevGeom& g, const DevModelPtrs& m, CellCache& C, int key) {
  if (key == C.key) return;
  C.key = key;
  const int s1 = g.n2p, s0 = g.n1 * g.n2p;
  const float4* p = m.nfg + key;
  const float* t = m.te + key;
  const int off[8] = {0, 1, s1, s1 + 1, s0, s0 + 1, s0 + s1, s0 + s1 + 1};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    C.c[k * kWaveLanes] = p[off[k]];
    C.t[k * kWaveLanes] = t[off[k]];
  }
}

__device__ __forceinline__ void weights8(float u, float v, float w, float W[8]) {
  const float u0 = 1.0f - u, v0 = 1.0f - v, w0 = 1.0f - w;
  const float a00 = u0 * v0, a01 = u0 * v, a10 = u * v0, a11 = u * v;
  W[0] = a00 * w0; W[1] = a00 * w; W[2] = a01 * w0; W[3] = a01 * w;
  W[4] = a10 * w0; W[5] = a10 * w; W[6] = a11 * w0; W[7] = a11 * w;
}

// n_e and grad n_e [cm^-3 / R_sun] at a point.
template <int KIND>
__device__ __forceinline__ void eval_grad(const DevGeom& g, const DevModelPtrs& m, CellCache& C, const StepOrigin& O,
                                          float dx, float dy, float dz, float& ne, float& gx, float& gy, float& gz) {
  Loc L;
  locate<KIND>(g, O, dx, dy, dz, L);
  ensure_cell(g, m, C, L.key);
  float W[8];
  weights8(L.u, L.v, L.w, W);
  float n = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 q = C.c[k * kWaveLanes];
    n += W[k] * q.x;
    G0 += W[k] * q.y;
    G1 += W[k] * q.z;
    G2 += W[k] * q.w;
  }
  // Clamped edges keep the edge vertex's gradient: the force is continuous there.
  ne = n;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    // grad = G0/(r dl) r_hat + G1/(r dth) theta_hat + G2/(r sin(theta) dphi) phi_hat
    const float gr = G0 * g.inv_dl * L.rinv;
    const float gt = G1 * g.inv_dth * L.rinv;
    const float ct = L.z * L.rinv, st = L.rho * L.rinv;
    const float cph = L.axis ? 1.0f : L.x * L.rhoinv;
    const float sph = L.axis ? 0.0f : L.y * L.rhoinv;
    const float gp = L.axis ? 0.0f : G2 * g.inv_dph * L.rhoinv;
    const float grr = gr * L.rinv;
    gx = grr * L.x + gt * ct * cph - gp * sph;
    gy = grr * L.y + gt * ct * sph + gp * cph;
    gz = grr * L.z - gt * st;
  } else {
    gx = G0 * g.inv_sp[0];
    gy = G1 * g.inv_sp[1];
    gz = G2 * g.inv_sp[2];
  }
}

// n_e and T at a point (values only).
template <int KIND>
__device__ __forceinline__ void eval_value(const DevGeom& g, const DevModelPtrs& m, CellCache& C, const StepOrigin& O,
                                           float dx, float dy, float dz, float& ne, float& te) {
  Loc L;
  locate<KIND>(g, O, dx, dy, dz, L);
  ensure_cell(g, m, C, L.key);
  float W[8];
  weights8(L.u, L.v, L.w, W);
  float n = 0.f, t = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    n += W[k] * C.c[k * kWaveLanes].x;
    t += W[k] * C.t[k * kWaveLanes];
  }
  ne = n;
  te = t;
}

struct RayState {
  double rx, ry, rz;                 // position r_i (FP64 accumulator)
  double px, py, pz;                 // normalised wavevector p_i (FP64 accumulator)
  double A, P;                       // composite: emitted part, transmittance (front to back)
  double tau, lns, s_arc;
  float rmin;
  int n;                             // steps taken
  int id;                            // flat ray index
  int model;
  float cf;                          // -1/2 Xf, Xf = (8.98e3 / f)^2
  double cfd;                        // the same in FP64 (applied to the accumulated increments)
  float xff;                         // Xf
  float f2, lnf;                     // f^2, ln f
  double f;
  int path_slot, path_len;
};

// Chord-sphere crossing: root in [0, 1] of |o + lam d|^2 = R^2 (outward: larger root).
template <class Real>
__device__ __forceinline__ Real crossing(Real ox, Real oy, Real oz, Real dx, Real dy, Real dz, double R, bool outward) {
  const Real A = dx * dx + dy * dy + dz * dz;
  const Real B = ox * dx + oy * dy + oz * dz;
  const Real Cc = ox * ox + oy * oy + oz * oz - Real(R * R);
  const Real D = B * B - A * Cc;
  if (!(D >= Real(0))) return Real(1);
  const Real s = sqrt(D);
  Real lam;
  if (outward) lam = (B <= Real(0)) ? (-B + s) / A : -Cc / (B + s);
  else lam = (B < Real(0)) ? Cc / (-B + s) : (-B - s) / A;
  if (!(lam > Real(0))) lam = Real(0);
  if (lam > Real(1)) lam = Real(1);
  return lam;
}

__device__ __forceinline__ int find_path_slot(const TraceArgs& a, int id) {
  int lo = 0, hi = a.n_path - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = a.path_rays[mid];
    if (v == id) return mid;
    if (v < id) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// Ray index -> (image, pixel) for the image layout [model][freq][nv][nu].
__device__ __forceinline__ void ray_coords(const TraceArgs& a, int id, int& model, int& fi, int& i, int& j) {
  const int npx = a.nu * a.nv;
  const int img = id / npx;
  const int px = id - img * npx;
  model = img / a.n_freq;
  fi = img - model * a.n_freq;
  i = px / a.nu;
  j = px - i * a.nu;
}

// A ray that misses the model: T_b = tb_sky; its "exit" is its pixel point in the
// image plane through the Sun's centre.
__device__ __forceinline__ void write_miss(const TraceArgs& a, int id, double b, double px, double py, double pz) {
  a.tb[id] = float(a.tb_sky);
  if (a.info) {
    rt_ray_info inf;
    inf.n_steps = 0; inf.code = kMiss; inf.flags = 0; inf._pad[0] = inf._pad[1] = 0;
    inf.exit_pos[0] = float(px); inf.exit_pos[1] = float(py); inf.exit_pos[2] = float(pz);
    inf.tau = 0.f; inf.ln_s_end = 0.f; inf.r_min = float(b);
    a.info[id] = inf;
  }
}

// Launch (Sec. 3.2): start on the r_max sphere, direction -o, p0 = n(r0) (-o).
// Returns false for a ray that misses the model (output written).
template <int KIND>
__device__ bool init_ray(const TraceArgs& a, int id, RayState& R, CellCache& C) {
  int model, fi, i, j;
  ray_coords(a, id, model, fi, i, j);
  const double pu = -a.half_u + (j + 0.5) * 2.0 * a.half_u / a.nu;
  const double pv = -a.half_v + (i + 0.5) * 2.0 * a.half_v / a.nv;
  const double b2 = pu * pu + pv * pv;
  const double rmax = a.g.r_max;
  if (b2 >= rmax * rmax) {
    write_miss(a, id, sqrt(b2), pu * a.u[0] + pv * a.v[0], pu * a.u[1] + pv * a.v[1], pu * a.u[2] + pv * a.v[2]);
    return false;
  }
  const double x0 = sqrt(rmax * rmax - b2);
  const double r0x = x0 * a.o[0] + pu * a.u[0] + pv * a.v[0];
  const double r0y = x0 * a.o[1] + pu * a.u[1] + pv * a.v[1];
  const double r0z = x0 * a.o[2] + pu * a.u[2] + pv * a.v[2];
  R.rx = r0x; R.ry = r0y; R.rz = r0z;
  C.key = -1;  // the lane's cached cell may belong to another model
  const double f = a.freqs[fi];
  const double xf = (8.98e3 / f) * (8.98e3 / f);
  R.f = f;
  R.xff = float(xf);
  R.cf = float(-0.5 * xf);
  R.cfd = -0.5 * xf;
  R.f2 = float(f * f);
  R.lnf = float(log(f));
  R.model = model;
  R.id = id;
  double nidx = 1.0;
  if (a.flags & RT_USE_REFRACTION) {
    float ne, te;
    StepOrigin O;
    make_origin<KIND>(a.g, r0x, r0y, r0z, O);
    eval_value<KIND>(a.g, a.models[model], C, O, 0.f, 0.f, 0.f, ne, te);
    const float n2 = 1.0f - R.xff * ne;
    nidx = n2 > 0.f ? double(sqrtf(n2)) : 0.0;
  }
  R.px = -nidx * a.o[0]; R.py = -nidx * a.o[1]; R.pz = -nidx * a.o[2];
  R.A = 0.0; R.P = 1.0; R.tau = 0.0; R.lns = 0.0; R.s_arc = 0.0;
  R.rmin = float(rmax);
  R.n = 0;
  R.path_slot = (a.n_path > 0) ? find_path_slot(a, id) : -1;
  R.path_len = 0;
  return true;
}

template <class Real>
__device__ __forceinline__ void finish_ray(const TraceArgs& a, const RayState& R, int code, Real ex, Real ey, Real ez,
                                           Real lam) {
  const double tbc = (code == kHit) ? a.tb_inner : a.tb_sky;
  const double tb = R.A + R.P * tbc;
  a.tb[R.id] = float(tb);
  if (a.info) {
    rt_ray_info inf;
    inf.n_steps = R.n;
    inf.code = int8_t(code);
    inf.flags = ((code == kExit || code == kHit) && (lam < Real(1e-4) || lam > Real(1) - Real(1e-4)))
                    ? int8_t(RT_RAY_FLAG_MARGINAL) : int8_t(0);
    inf._pad[0] = inf._pad[1] = 0;
    inf.exit_pos[0] = float(ex); inf.exit_pos[1] = float(ey); inf.exit_pos[2] = float(ez);
    inf.tau = float(R.tau);
    inf.ln_s_end = float(R.lns);
    const float re = float(sqrt(ex * ex + ey * ey + ez * ez));
    inf.r_min = fminf(R.rmin, re);
    a.info[R.id] = inf;
  }
  if (R.path_slot >= 0) a.path_len[R.path_slot] = R.path_len;
}

// One central RK4 step with its two perturbed retraces, termination test and
// transfer segment.  Returns the termination code (kRunning to continue).
template <bool MIXED, int KIND>
__device__ int ray_step(const TraceArgs& a, RayState& R, CellCache& C) {
  using Real = typename RealOf<MIXED>::T;
  const DevModelPtrs& M = a.models[R.model];
  const bool refr = (a.flags & RT_USE_REFRACTION) != 0;
  const bool mag = refr && (a.flags & RT_USE_MAGNIFICATION) != 0;

  // All evaluation points of this step are r_i + (FP32 offset); forces and stage
  // offsets are FP32, the state r_i, p_i accumulates in FP64.
  StepOrigin O;
  make_origin<KIND>(a.g, R.rx, R.ry, R.rz, O);
  const float pxf = float(R.px), pyf = float(R.py), pzf = float(R.pz);
  float h;
  double hd;
  double drx, dry, drz, dpx = 0.0, dpy = 0.0, dpz = 0.0;
  float d2x = 0.f, d2y = 0.f, d2z = 0.f, d3x = 0.f, d3y = 0.f, d3z = 0.f;
  float F1x = 0.f, F1y = 0.f, F1z = 0.f, F2x = 0.f, F2y = 0.f, F2z = 0.f, F3x = 0.f, F3y = 0.f, F3z = 0.f;
  if (refr) {
    // Stage 1 at r_i also sets the step: dt = ds_max / max(n(r_i), n_floor).
    float ne, g1x, g1y, g1z, gx, gy, gz;
    eval_grad<KIND>(a.g, M, C, O, 0.f, 0.f, 0.f, ne, g1x, g1y, g1z);
    F1x = R.cf * g1x; F1y = R.cf * g1y; F1z = R.cf * g1z;
    const float n2 = 1.0f - R.xff * ne;
    const float ni = n2 > 0.f ? sqrtf(n2) : 0.f;
    // the FP64 step enters the state update; its FP32 rounding drives the stages
    hd = (ni > a.n_floor) ? a.ds_max_d / double(ni) : a.ds_max_d / a.n_floor_d;
    h = float(hd);
    const float hh = 0.5f * h;
    d2x = hh * pxf; d2y = hh * pyf; d2z = hh * pzf;
    float g2x, g2y, g2z;
    eval_grad<KIND>(a.g, M, C, O, d2x, d2y, d2z, ne, g2x, g2y, g2z);
    F2x = R.cf * g2x; F2y = R.cf * g2y; F2z = R.cf * g2z;
    d3x = hh * (pxf + hh * F1x); d3y = hh * (pyf + hh * F1y); d3z = hh * (pzf + hh * F1z);
    float g3x, g3y, g3z;
    eval_grad<KIND>(a.g, M, C, O, d3x, d3y, d3z, ne, g3x, g3y, g3z);
    F3x = R.cf * g3x; F3y = R.cf * g3y; F3z = R.cf * g3z;
    const float d4x = h * (pxf + hh * F2x), d4y = h * (pyf + hh * F2y), d4z = h * (pzf + hh * F2z);
    eval_grad<KIND>(a.g, M, C, O, d4x, d4y, d4z, ne, gx, gy, gz);
    // RK4: dr = h p + h^2/6 (F1 + F2 + F3), dp = h/6 (F1 + 2 F2 + 2 F3 + F4),
    // F = -1/2 Xf grad n_e with the coefficient applied in FP64.
    const double c6 = R.cfd * hd * (1.0 / 6.0);
    drx = hd * R.px + hd * c6 * double(g1x + g2x + g3x);
    dry = hd * R.py + hd * c6 * double(g1y + g2y + g3y);
    drz = hd * R.pz + hd * c6 * double(g1z + g2z + g3z);
    dpx = c6 * double(g1x + 2.f * g2x + 2.f * g3x + gx);
    dpy = c6 * double(g1y + 2.f * g2y + 2.f * g3y + gy);
    dpz = c6 * double(g1z + 2.f * g2z + 2.f * g3z + gz);
  } else {
    // Straight line of sight: no force, |p| = 1, dt = ds_max.
    h = a.ds_max;
    hd = a.ds_max_d;
    drx = a.ds_max_d * R.px; dry = a.ds_max_d * R.py; drz = a.ds_max_d * R.pz;
  }
  if (!(isfinite(drx) && isfinite(dry) && isfinite(drz) && isfinite(dpx) && isfinite(dpy) && isfinite(dpz))) {
    R.n += 1;
    finish_ray<Real>(a, R, kNonfinite, Real(R.rx), Real(R.ry), Real(R.rz), Real(1));
    return kNonfinite;
  }

  // Eq. 5: chord direction (the chord is exactly the increment dr).
  const Real dx = Real(drx), dy = Real(dry), dz = Real(drz);
  const Real ds = sqrt(dx * dx + dy * dy + dz * dz);
  Real lnM = Real(0);
  if (mag) {
    const Real tx = dx / ds, ty = dy / ds, tz = dz / ds;
    // Eq. 6: a = z unless |t_z| is near 1, then y; e1 = a x t / |a x t|, e2 = t x e1.
    Real c1x, c1y, c1z;
    if (fabs(tz) > Real(0.9)) { c1x = tz; c1y = Real(0); c1z = -tx; }
    else { c1x = -ty; c1y = tx; c1z = Real(0); }
    const Real ci = Real(1) / sqrt(c1x * c1x + c1y * c1y + c1z * c1z);
    const Real e1x = c1x * ci, e1y = c1y * ci, e1z = c1z * ci;
    const Real e2x = ty * e1z - tz * e1y, e2y = tz * e1x - tx * e1z, e2z = tx * e1y - ty * e1x;
    const Real eps = Real(a.eta) * ds;  // Eq. 8
    // Eqs. 7 and 9 in difference form: the perturbed ray starts at r_i + eps e_j with
    // the central wavevector; its RK4 end point minus the central one is
    // eps e_j + h^2/6 (dF1 + dF2 + dF3), dF_k the force differences at the first
    // three stages (the fourth stage only moves p, which is discarded).
    Real sep[2][3];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const Real ex = jj == 0 ? e1x : e2x, ey = jj == 0 ? e1y : e2y, ez = jj == 0 ? e1z : e2z;
      const Real d0x = eps * ex, d0y = eps * ey, d0z = eps * ez;
      const float fx = float(d0x), fy = float(d0y), fz = float(d0z);
      const float hh = 0.5f * h;
      float ne, gx, gy, gz;
      eval_grad<KIND>(a.g, M, C, O, fx, fy, fz, ne, gx, gy, gz);
      const float q1x = R.cf * gx - F1x, q1y = R.cf * gy - F1y, q1z = R.cf * gz - F1z;
      eval_grad<KIND>(a.g, M, C, O, d2x + fx, d2y + fy, d2z + fz, ne, gx, gy, gz);
      const float q2x = R.cf * gx - F2x, q2y = R.cf * gy - F2y, q2z = R.cf * gz - F2z;
      const float hq = hh * hh;
      eval_grad<KIND>(a.g, M, C, O, d3x + fx + hq * q1x, d3y + fy + hq * q1y, d3z + fz + hq * q1z, ne, gx, gy, gz);
      const float q3x = R.cf * gx - F3x, q3y = R.cf * gy - F3y, q3z = R.cf * gz - F3z;
      const float hh6 = h * h * (1.0f / 6.0f);
      sep[jj][0] = d0x + Real(hh6 * (q1x + q2x + q3x));
      sep[jj][1] = d0y + Real(hh6 * (q1y + q2y + q3y));
      sep[jj][2] = d0z + Real(hh6 * (q1z + q2z + q3z));
    }
    // Eqs. 10-11: M = |(dr1 x dr2) . t| / eps^2.
    const Real cx = sep[0][1] * sep[1][2] - sep[0][2] * sep[1][1];
    const Real cy = sep[0][2] * sep[1][0] - sep[0][0] * sep[1][2];
    const Real cz = sep[0][0] * sep[1][1] - sep[0][1] * sep[1][0];
    const Real area = fabs(cx * tx + cy * ty + cz * tz);
    lnM = log(area / (eps * eps));
  }

  // Termination on the two spheres, last chord truncated at the crossing.
  const Real ox = Real(R.rx), oy = Real(R.ry), oz = Real(R.rz);
  const Real nx = ox + dx, ny = oy + dy, nz = oz + dz;
  const Real r1sq = nx * nx + ny * ny + nz * nz;
  int code = kRunning;
  Real lam = Real(1);
  if (a.g.has_inner && r1sq <= Real(a.g.r_in * a.g.r_in)) {
    code = kHit;
    lam = crossing<Real>(ox, oy, oz, dx, dy, dz, a.g.r_in, false);
  } else if (r1sq >= Real(a.g.r_max * a.g.r_max) && R.n >= 1) {
    code = kExit;
    lam = crossing<Real>(ox, oy, oz, dx, dy, dz, a.g.r_max, true);
  } else if (R.n + 1 == a.max_steps) {
    code = kMaxSteps;
  }

  // Segment at the chord midpoint: free-free kappa*n, dtau = kappa*n R_sun lam dt,
  // gamma = -lam ln M (the d ln S/ds term over the segment, in the transfer direction).
  const float hl = 0.5f * float(lam);
  float ne_m, te_m;
  eval_value<KIND>(a.g, M, C, O, hl * float(drx), hl * float(dry), hl * float(drz), ne_m, te_m);
  Real dtau = Real(0);
  if (!(a.flags & RT_TEST_NO_ABSORPTION)) {
    const float lt = logf(te_m);
    const float lnl = (te_m >= 2.0e5f) ? 24.5f + lt - R.lnf : 18.2f + 1.5f * lt - R.lnf;
    const float kn = kFFCoefF * ne_m * ne_m * lnl / (R.f2 * te_m * sqrtf(te_m));
    dtau = Real(kn) * Real(kRsunCm) * lam * Real(hd);
  }
  const Real gamma = -(lam * lnM);
  const Real xs = dtau + gamma;
  const Real em = expm1(-xs);
  const Real phi = (xs == Real(0)) ? Real(1) : -em / xs;
  R.A += R.P * double(Real(te_m) * dtau * phi);
  R.P *= double(Real(1) + em);
  R.tau += double(dtau);
  R.lns += double(lam * lnM);
  R.s_arc += double(lam * ds);
  R.n += 1;

  if (R.path_slot >= 0 && R.path_len < a.path_cap) {
    float* rec = a.path_out + (size_t(R.path_slot) * a.path_cap + R.path_len) * kPathStride;
    rec[0] = float(ox + lam * dx); rec[1] = float(oy + lam * dy); rec[2] = float(oz + lam * dz);
    rec[3] = float(R.s_arc); rec[4] = float(lnM); rec[5] = float(lnM / ds);
    rec[6] = float(R.tau); rec[7] = ne_m; rec[8] = te_m;
    R.path_len += 1;
  }

  if (code != kRunning) {
    finish_ray<Real>(a, R, code, ox + lam * dx, oy + lam * dy, oz + lam * dz, lam);
    return code;
  }
  R.rx += drx; R.ry += dry; R.rz += drz;
  R.px += dpx; R.py += dpy; R.pz += dpz;
  const float rr = float(sqrt(R.rx * R.rx + R.ry * R.ry + R.rz * R.rz));
  R.rmin = fminf(R.rmin, rr);
  return kRunning;
}

}  // namespace rt
