// Per-ray device code: model gathers, one RK4 step with step-wise perturbation
// retracing, free-free segment transfer, launch and finish.
//
// Paper: "Modeling the Thermal Low-Frequency Radio Sun with Ray Tracing".
//   Ray equations: Sec. 2.1, Eq. 4, in the normalised form dr/dt = p,
//   dp/dt = -1/2 grad X with X = (8.98e3)^2 n_e / f^2 (|p| = n, ds = n dt).
//   Perturbation retracing and magnification: Eqs. 5-11 (area without the 1/2).
//   Transfer with the geometric term: Eqs. 2-3, 12; one exact exponential
//   update per segment, composited front to back (the same products as the
//   back-to-front solution of Sec. 3.2).
//   Free-free: Rayleigh-Jeans closed form with the two-branch Coulomb
//   logarithm of Dulk (1985).
//
// Precision: every evaluation of the model (position offsets, coordinates,
// trilinear gathers, forces) is FP32.  Three variants of the rest:
//   default       the ray state r_i, p_i, the step increments and the grid index
//                 of r_i in FP64; ray-tube area and the optical depth /
//                 brightness accumulators in FP64;
//   FP32 stepping the ray state, increments and grid index (integer cell + FP32
//                 fraction) in FP32; area and accumulators in FP64;
//   all-FP32      everything in FP32.
#pragma once

#include <type_traits>

#include "rt_internal.hpp"

namespace rt {

constexpr double kRsunCm = 6.957e10;
constexpr float kFFCoefF = 9.78e-3f;
constexpr float kPiF = 3.14159265358979323846f;

enum : int { kRunning = 0, kExit = 1, kHit = 2, kMiss = 3, kMaxSteps = 4, kNonfinite = 5 };

template <bool MIXED> struct RealOf { using T = double; };
template <> struct RealOf<false> { using T = float; };

// Precision variants of the trace kernels.
enum : int { kPrecDefault = 0, kPrecFp32Step = 1, kPrecFp32 = 2 };

// ---------------------------------------------------------------------------
// Small math kernels with few constants (so that nothing large is kept live
// across the step loop).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// Odd Taylor series of atan on |t| <= tan(pi/8): truncation below 2e-8.
__device__ __forceinline__ float atan_poly(float t) {
  const float t2 = t * t;
  float s = 1.0f / 15.0f;
  s = fmaf(s, -t2, 1.0f / 13.0f);
  s = fmaf(s, -t2, 1.0f / 11.0f);
  s = fmaf(s, -t2, 1.0f / 9.0f);
  s = fmaf(s, -t2, 1.0f / 7.0f);
  s = fmaf(s, -t2, 1.0f / 5.0f);
  s = fmaf(s, -t2, 1.0f / 3.0f);
  s = fmaf(s, -t2, 1.0f);
  return t * s;
}

// atan2 in FP32: octant reduction to [0, 1], then atan(a) = pi/4 + atan((a-1)/(a+1))
// above tan(pi/8), then the series.  Absolute error below 3e-8 rad.
__device__ __forceinline__ float fast_atan2f(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float q = mx > 0.0f ? mn * rcpf(mx) : 0.0f;
  const bool red = q > 0.41421356f;
  const float t = red ? (q - 1.0f) * rcpf(q + 1.0f) : q;
  float r = atan_poly(t) + (red ? 0.25f * kPiF : 0.0f);
  if (ay > ax) r = 0.5f * kPiF - r;
  if (x < 0.0f) r = kPiF - r;
  return copysignf(r, y);
}

// Angle of a small increment: atan2(y, x) for x > 0 and |y| <= x / 10 is
// t - t^3/3 + t^5/5 - t^7/7 with t = y / x (truncation below 1.2e-9 of the
// angle); any other argument goes through fast_atan2f.  The angular increments
// from a step's origin to its evaluation points are this small except next to
// the polar axis.
__device__ __forceinline__ float atan2_inc(float y, float x) {
  if (x > 0.0f && fabsf(y) <= 0.1f * x) {
    const float t = y * rcpf(x), t2 = t * t;
    float s = -1.0f / 7.0f;
    s = fmaf(s, t2, 1.0f / 5.0f);
    s = fmaf(s, t2, -1.0f / 3.0f);
    return fmaf(t * t2, s, t);
  }
  return fast_atan2f(y, x);
}

// log1p in FP32: 2 atanh(z / (2 + z)) by its odd series for |z| <= 1/4
// (relative truncation below 1e-10); log2 instruction otherwise.
__device__ __forceinline__ float fast_log1pf(float z) {
  if (fabsf(z) <= 0.25f) {
    const float w = z * rcpf(2.0f + z);
    const float w2 = w * w;
    float s = 1.0f / 9.0f;
    s = fmaf(s, w2, 1.0f / 7.0f);
    s = fmaf(s, w2, 1.0f / 5.0f);
    s = fmaf(s, w2, 1.0f / 3.0f);
    s = fmaf(s, w2, 1.0f);
    return 2.0f * w * s;
  }
  return __builtin_amdgcn_logf(1.0f + z) * 0.69314718056f;
}

// log1p for the small radius increments of the evaluation points: the Taylor
// series to z^7 in Horner form for |z| <= 1/20 (relative truncation below
// 5e-12; no reciprocal), fast_log1pf otherwise.
__device__ __forceinline__ float log1p_inc(float z) {
  if (fabsf(z) <= 0.05f) {
    float q = 1.0f / 7.0f;
    q = fmaf(q, z, -1.0f / 6.0f);
    q = fmaf(q, z, 1.0f / 5.0f);
    q = fmaf(q, z, -1.0f / 4.0f);
    q = fmaf(q, z, 1.0f / 3.0f);
    q = fmaf(q, z, -1.0f / 2.0f);
    q = fmaf(q, z, 1.0f);
    return z * q;
  }
  return fast_log1pf(z);
}

// FP64 reciprocal: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// Square roots without the correctly rounded expansion the compiler emits for
// sqrt(): FP32 with the hardware instruction (about 1 ulp), FP64 as x rsqrt(x)
// with the hardware estimate refined by two Newton steps (full FP64 accuracy,
// not correctly rounded).  0 for x <= 0.
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
// Reciprocal square root with the hardware instruction: rsqrtf() adds a
// rescaling for denormal arguments, which the radii and cylinder radii it is
// used for never are (the same result otherwise).
__device__ __forceinline__ float rsqrt_fast(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double sqrt64(double x) { return x > 0.0 ? x * rsqrt64(x) : 0.0; }
// The same for the precision of the ray-tube area (double, or float in the
// all-FP32 variant).
__device__ __forceinline__ double rsqrt_r(double x) { return rsqrt64(x); }
__device__ __forceinline__ float rsqrt_r(float x) { return rsqrt_fast(x); }
__device__ __forceinline__ double rcp_r(double x) { return rcp64(x); }
__device__ __forceinline__ float rcp_r(float x) { return rcpf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt64(x); }
__device__ __forceinline__ float sqrt_r(float x) { return x > 0.0f ? sqrt_fast(x) : 0.0f; }

// FP64 series for the per-step index increments, valid for small arguments
// only (|w|, |t| <= 1/32): three shared coefficients keep the loop free of
// FP64 constants that the compiler would pin in registers.
// log1p(z) = 2 atanh(w), w = z / (2 + z): truncation w^9/9 < 4e-15 relative.
__device__ __forceinline__ double log1p_small64(double z) {
  const double w = z * rcp64(2.0 + z);
  const double w2 = w * w;
  const double s = fma(fma(fma(1.0 / 7.0, w2, 1.0 / 5.0), w2, 1.0 / 3.0), w2, 1.0);
  return 2.0 * w * s;
}
// atan(t) = t (1 - t^2/3 + t^4/5 - t^6/7): truncation t^8/9 < 1e-13 relative.
__device__ __forceinline__ double atan_small64(double t) {
  const double t2 = t * t;
  const double s = fma(fma(fma(-1.0 / 7.0, t2, 1.0 / 5.0), t2, -1.0 / 3.0), t2, 1.0);
  return t * s;
}
constexpr double kSmall64 = 1.0 / 32.0;

// General FP64 atan2 and log for the rare large increments, built on the same
// series: atan(t) = 2 atan(t / (1 + sqrt(1 + t^2))) halves the argument until
// |t| <= 1/32, log(x) = 2 log(sqrt(x)) until |x - 1| <= 1/32.
__device__ __forceinline__ double atan2_64(double y, double x) {
  if (x == 0.0 && y == 0.0) return 0.0;
  const bool flip = x < 0.0;
  const double ax = flip ? -x : x;
  double t = fabs(y) > ax * 1e12 ? 1e12 : y * rcp64(ax);
  double scale = 1.0;
  while (fabs(t) > kSmall64) {
    t = t * rcp64(1.0 + sqrt(fma(t, t, 1.0)));
    scale *= 2.0;
  }
  double r = scale * atan_small64(t);  // in (-pi/2, pi/2)
  if (flip) r = (y >= 0.0 ? 3.141592653589793238463 : -3.141592653589793238463) - r;
  return r;
}
__device__ __forceinline__ double log_64(double x) {
  double scale = 1.0;
  while (fabs(x - 1.0) > kSmall64) {
    x = sqrt(x);
    scale *= 2.0;
  }
  return scale * log1p_small64(x - 1.0);
}

// Library FP64 functions, kept out of line: used at ray start and when an
// incremental index update leaves its series range (rare).
__device__ __noinline__ double lib_log(double x) { return log(x); }
__device__ __noinline__ double lib_atan2(double y, double x) { return atan2(y, x); }

// ---------------------------------------------------------------------------
// Per-lane cell cache in LDS: the 8 corners of the last cell a lane touched,
// (n_e, index-space gradient) and T of corner k = 4 i + 2 j + k' for offsets
// (i, j, k') along axes 0, 1, 2.  Slots are corner-major ([corner][lane]) so
// that the 64 lanes of a wave read consecutive 16-byte words (no bank
// conflicts).  Each lane only reads its own slots, which it wrote itself; LDS
// operations of a wave complete in order.
// ---------------------------------------------------------------------------
struct CellCache {
  int key;
  float4* c;  // LDS, corner k at c[k * kWaveLanes]
  float* t;   // LDS, corner k at t[k * kWaveLanes]
};

__device__ __forceinline__ void ensure_cell(const DevGeom& g, const float4* nfg, const float* te, CellCache& C,
                                            int key) {
  if (key == C.key) return;
  C.key = key;
  const int s1 = g.n2p, s0 = g.n1 * g.n2p;
  const int off[4] = {0, s1, s0, s0 + s1};
  // two corners (one 32-byte run along axis 2) at a time keeps few values live
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4 a0 = nfg[key + off[k]], a1 = nfg[key + off[k] + 1];
    const float t0 = te[key + off[k]], t1 = te[key + off[k] + 1];
    C.c[(2 * k) * kWaveLanes] = a0;
    C.c[(2 * k + 1) * kWaveLanes] = a1;
    C.t[(2 * k) * kWaveLanes] = t0;
    C.t[(2 * k + 1) * kWaveLanes] = t1;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ---------------------------------------------------------------------------
// Grid index bookkeeping.  The continuous grid index of a step's origin r_i is
// carried in FP64 and advanced incrementally with cancellation-free small-offset
// formulas; every evaluation point r_i + d (d a small FP32 offset) then gets its
// index as the origin's (integer, FP32 fraction) plus an FP32 increment.  FP32
// alone cannot place a point inside a cell to better than ulp(r)/(r dl), about
// 1e-6..5e-6 of a cell, which perturbs every force by ~1e-6 and moves the exit
// point of a strongly refracted ray by ~1e-4 R_sun.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ void index_exact(const DevGeom& g, double X, double Y, double Z, double& b0, double& b1,
                                            double& b2) {
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    const double rho2 = X * X + Y * Y;
    const double r2 = rho2 + Z * Z;
    b0 = (0.5 * lib_log(r2) - g.ln_rin_d) * g.inv_dl_d;
    b1 = lib_atan2(sqrt(rho2), Z) * g.inv_dth_d - 0.5;
    double ph = rho2 > 0.0 ? lib_atan2(Y, X) : 0.0;
    if (ph < 0.0) ph += 6.283185307179586476925;
    b2 = ph * g.inv_dph_d;
    if (b2 >= double(g.n2)) b2 -= double(g.n2);
  } else {
    b0 = (X - g.org_d[0]) * g.inv_sp_d[0];
    b1 = (Y - g.org_d[1]) * g.inv_sp_d[1];
    b2 = (Z - g.org_d[2]) * g.inv_sp_d[2];
  }
}

struct StepOrigin {
  float x, y, z;        // r_i in FP32 (for the offset formulas)
  float r2, inv_r2, rho2, rho;
  int i0, i1, i2;       // integer part of r_i's grid index
  float f0, f1, f2;     // fractional part in [0, 1)
};

__device__ __forceinline__ void split_index(double b, int& i, float& f) {
  double fl = floor(b);
  if (!(fl >= -1.0e9 && fl <= 1.0e9)) fl = 0.0;  // NaN guard
  i = int(fl);
  f = float(b - fl);
}

struct Loc {
  int key;
  float u, v, w;
  // chain-rule pieces at the evaluation point (spherical)
  float rinv, rhoinv, rho, x, y, z;
  float axz;           // z on the polar axis, else 0
  bool axis;
  bool cl0, cl1, cl2;  // index held at an edge along axis 0, 1, 2 (no dependence on position)
};

// Cell of a clamped axis from (integer base, FP32 index offset): a in [0, n-2],
// u in [0, 1]; beyond an edge the index is held at the edge.
__device__ __forceinline__ void cell_clamped(float x, int I, int n, int& a, float& u, bool& held) {
  float fk = floorf(x);
  if (!(fk >= -1.0e9f && fk <= 1.0e9f)) fk = 0.0f;  // NaN guard keeps every gather in bounds
  u = x - fk;
  a = I + int(fk);
  held = false;
  if (a < 0) { a = 0; u = 0.0f; held = true; }
  else if (a > n - 2) { a = n - 2; u = 1.0f; held = true; }
}

// Periodic axis: the offset of an evaluation point from its step origin is an
// angle in [-pi, pi], at most n/2 cells, so one wrap in either direction brings
// the cell into [0, n); anything else (a non-finite offset) is sent to cell 0.
__device__ __forceinline__ void cell_periodic(float x, int I, int n, int& c, float& w) {
  float fk = floorf(x);
  if (!(fk >= -1.0e9f && fk <= 1.0e9f)) fk = 0.0f;
  w = x - fk;
  c = I + int(fk);
  if (c >= n) c -= n;
  else if (c < 0) c += n;
  if ((unsigned)c >= (unsigned)n) c = 0;
}

// AT_ORIGIN: the point is r_i itself (d = 0), whose index is the origin's and
// whose chain-rule pieces need no offset arithmetic (the same values as the
// general form at d = 0).
template <int KIND, bool AT_ORIGIN = false>
__device__ __forceinline__ void locate(const DevGeom& g, const StepOrigin& O, float dx, float dy, float dz, Loc& L) {
  float x0, x1, x2;
  if constexpr (AT_ORIGIN) {
    x0 = O.f0; x1 = O.f1; x2 = O.f2;
    if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
      const float m = fmaxf(O.rho2, 0.0f);
      const float rhoi = m > 1.0e-24f ? rsqrt_fast(m) : 0.0f;
      const float rhoq = m * rhoi;
      L.rinv = rsqrt_fast(O.r2);
      L.rho = rhoq;
      L.axis = rhoq < 1e-12f;
      L.rhoinv = L.axis ? 0.0f : rhoi;
      L.x = O.x; L.y = O.y; L.z = O.z;
      L.axz = L.axis ? O.z : 0.0f;
    }
  } else if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    // radius: |q|^2 = |r_i|^2 (1 + c / |r_i|^2), c = 2 r_i.d + |d|^2
    const float rd = O.x * dx + O.y * dy;
    const float dd = dx * dx + dy * dy;
    const float c = 2.0f * (rd + O.z * dz) + (dd + dz * dz);
    x0 = O.f0 + 0.5f * log1p_inc(c * O.inv_r2) * g.inv_dl;
    // azimuth: angle from (x_i, y_i) to (x_i + dx, y_i + dy)
    x2 = O.f2 + atan2_inc(O.x * dy - O.y * dx, O.rho2 + rd) * g.inv_dph;
    // colatitude: angle from (z_i, rho_i) to (z_q, rho_q) in the meridional plane
    const float e = 2.0f * rd + dd;
    const float m = fmaxf(O.rho2 + e, 0.0f);
    const float rhoi = m > 1.0e-24f ? rsqrt_fast(m) : 0.0f;  // 0 on the polar axis (rho < 1e-12)
    const float rhoq = m * rhoi;
    const float den = rhoq + O.rho;
    const float zq = O.z + dz;
    // the angle between (z_i, rho_i) and (z_q, rho_q) from its sine and cosine
    // parts, both scaled by rho_q + rho_i > 0 (which leaves the angle as it is)
    // so that rho_q - rho_i = e / (rho_q + rho_i) needs no division; on the
    // axis both parts vanish
    x1 = O.f1 + atan2_inc(O.z * e - O.rho * dz * den, den * (O.z * zq + O.rho * rhoq)) * g.inv_dth;
    L.rinv = rsqrt_fast(O.r2 + c);
    L.rho = rhoq;
    L.axis = rhoq < 1e-12f;
    L.rhoinv = L.axis ? 0.0f : rhoi;
    L.x = O.x + dx; L.y = O.y + dy; L.z = zq;
    L.axz = L.axis ? zq : 0.0f;
  } else {
    x0 = O.f0 + dx * g.inv_sp[0];
    x1 = O.f1 + dy * g.inv_sp[1];
    x2 = O.f2 + dz * g.inv_sp[2];
  }
  int a, b, c;
  cell_clamped(x0, O.i0, g.n0, a, L.u, L.cl0);
  cell_clamped(x1, O.i1, g.n1, b, L.v, L.cl1);
  L.cl2 = false;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) cell_periodic(x2, O.i2, g.n2, c, L.w);
  else cell_clamped(x2, O.i2, g.n2, c, L.w, L.cl2);
  // cell indices and grid extents are below 2^24 and keys below 2^31: 24-bit multiplies
  L.key = int(__umul24(__umul24(unsigned(a), unsigned(g.n1)) + unsigned(b), unsigned(g.n2p))) + c;
}

__device__ __forceinline__ void weights8(float u, float v, float w, float W[8]) {
  const float u0 = 1.0f - u, v0 = 1.0f - v, w0 = 1.0f - w;
  const float a00 = u0 * v0, a01 = u0 * v, a10 = u * v0, a11 = u * v;
  W[0] = a00 * w0; W[1] = a00 * w; W[2] = a01 * w0; W[3] = a01 * w;
  W[4] = a10 * w0; W[5] = a10 * w; W[6] = a11 * w0; W[7] = a11 * w;
}

// n_e and grad n_e [cm^-3 / R_sun] at r_i + d.  The gradient is the trilinear
// interpolant of the per-vertex index-space gradient (continuous across cell
// faces and clamped edges), mapped to Cartesian with the spherical unit vectors.
template <int KIND, bool AT_ORIGIN = false>
__device__ __forceinline__ void eval_grad(const DevGeom& g, const float4* nfg, const float* te, CellCache& C,
                                          const StepOrigin& O, float dx, float dy, float dz, float& ne, float& gx,
                                          float& gy, float& gz) {
  Loc L;
  locate<KIND, AT_ORIGIN>(g, O, dx, dy, dz, L);
  ensure_cell(g, nfg, te, C, L.key);
  float W[8];
  weights8(L.u, L.v, L.w, W);
  float n = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 q = C.c[k * kWaveLanes];
    n = fmaf(W[k], q.x, n);
    G0 = fmaf(W[k], q.y, G0);
    G1 = fmaf(W[k], q.z, G1);
    G2 = fmaf(W[k], q.w, G2);
    if (k == 3) __builtin_amdgcn_sched_barrier(0);
  }
  ne = n;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    // grad = G0/(r dl) r_hat + G1/(r dth) theta_hat + G2/(r sin(theta) dphi) phi_hat,
    // with r_hat = (x, y, z)/r, theta_hat = (z x/rho, z y/rho, -rho)/r and
    // phi_hat = (-y, x, 0)/rho collected over the Cartesian components:
    // g = x c - B y, y c + B x, grr z - A rho with A = G1/(r^2 dth),
    // B = G2/(rho^2 dphi), c = grr + A z/rho.  On the axis (1/rho taken as 0)
    // theta_hat is (cos theta, 0, -sin theta) and phi_hat drops out.
    const float r2i = L.rinv * L.rinv;
    const float grr = G0 * (g.inv_dl * r2i);
    const float A = G1 * (g.inv_dth * r2i);
    const float B = G2 * (g.inv_dph * (L.rhoinv * L.rhoinv));
    const float c = fmaf(A * L.z, L.rhoinv, grr);
    gx = fmaf(A, L.axz, fmaf(L.x, c, -B * L.y));
    gy = fmaf(L.y, c, B * L.x);
    gz = fmaf(grr, L.z, -A * L.rho);
  } else {
    gx = G0 * g.inv_sp[0];
    gy = G1 * g.inv_sp[1];
    gz = G2 * g.inv_sp[2];
  }
}

// n_e and T at r_i + d (values only).
template <int KIND, bool AT_ORIGIN = false>
__device__ __forceinline__ void eval_value(const DevGeom& g, const float4* nfg, const float* te, CellCache& C,
                                           const StepOrigin& O, float dx, float dy, float dz, float& ne, float& t) {
  Loc L;
  locate<KIND, AT_ORIGIN>(g, O, dx, dy, dz, L);
  ensure_cell(g, nfg, te, C, L.key);
  float W[8];
  weights8(L.u, L.v, L.w, W);
  float n = 0.f, tt = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    n = fmaf(W[k], C.c[k * kWaveLanes].x, n);
    tt = fmaf(W[k], C.t[k * kWaveLanes], tt);
  }
  ne = n;
  t = tt;
}

// ---------------------------------------------------------------------------
// Ray state and its life cycle.
// ---------------------------------------------------------------------------
// Grid index of r_i: the continuous index in FP64 (FP64 state), or the integer
// cell and the FP32 fraction in [0, 1) along each axis (FP32 state).
template <class S> struct GridIndexOf {
  double b0, b1, b2;
};
template <> struct GridIndexOf<float> {
  int i0, i1, i2;
  float fr0, fr1, fr2;
};

// S: position, wavevector and their step increments; Real: the ray-tube area
// and the transfer accumulators.
template <class S, class Real>
struct RayStateT : GridIndexOf<S> {
  S rx, ry, rz;             // position r_i (on termination: the end point)
  S px, py, pz;             // normalised wavevector p_i
  Real A;                   // composite: emitted part (front to back)
  Real lam_tot;             // optical depth of the segments so far, geometric term included
  Real tau, lns;
  S s_arc;
  double cfd;               // -1/2 Xf in FP64, Xf = (8.98e3 / f)^2
  const float4* nfg;        // this ray's model
  const float* te;
  float rmin, lam_end;
  float cf, xff, f2, lnf;
  int n;                    // steps taken
  int id;                   // flat ray index
  int code;
  int path_slot, path_len;
  // carried tube (kModeCarried only): separations of the two neighbour rays
  // from this ray at equal t, position and wavevector, and ln S at r_i
  double nb_r[2][3], nb_p[2][3];
  double tube_ln_s;
};
using RayState = RayStateT<double, double>;

template <int PREC> struct StateOf { using type = RayStateT<double, double>; };
template <> struct StateOf<kPrecFp32Step> { using type = RayStateT<float, double>; };
template <> struct StateOf<kPrecFp32> { using type = RayStateT<float, float>; };

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

template <int KIND, class S, class Real>
__device__ __forceinline__ void make_origin(const RayStateT<S, Real>& R, StepOrigin& O) {
  const S rho2 = R.rx * R.rx + R.ry * R.ry;
  const S r2 = rho2 + R.rz * R.rz;
  O.x = float(R.rx); O.y = float(R.ry); O.z = float(R.rz);
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    O.r2 = float(r2); O.inv_r2 = float(rcp_r(r2)); O.rho2 = float(rho2); O.rho = float(sqrt_r(rho2));
  } else {
    O.r2 = 0.f; O.inv_r2 = 0.f; O.rho2 = 0.f; O.rho = 0.f;
  }
  if constexpr (std::is_same<S, double>::value) {
    split_index(R.b0, O.i0, O.f0);
    split_index(R.b1, O.i1, O.f1);
    split_index(R.b2, O.i2, O.f2);
  } else {
    O.i0 = R.i0; O.i1 = R.i1; O.i2 = R.i2;
    O.f0 = R.fr0; O.f1 = R.fr1; O.f2 = R.fr2;
  }
}

// Advance the origin's grid index by the step increment d (FP64 small-offset
// formulas; exact recomputation outside their range).
template <int KIND>
__device__ __forceinline__ void index_advance(const DevGeom& g, RayState& R, double dx, double dy, double dz) {
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    const double X = R.rx, Y = R.ry, Z = R.rz;  // old origin
    const double rho2 = X * X + Y * Y, r2 = rho2 + Z * Z, rho = sqrt64(rho2);
    const double rd = X * dx + Y * dy;
    const double dd = dx * dx + dy * dy;
    const double c = 2.0 * (rd + Z * dz) + (dd + dz * dz);
    const double z = c * rcp64(r2);
    const double nX = X + dx, nY = Y + dy, nZ = Z + dz;
    if (fabs(z) <= kSmall64) R.b0 += 0.5 * log1p_small64(z) * g.inv_dl_d;
    else R.b0 = (0.5 * log_64(nX * nX + nY * nY + nZ * nZ) - g.ln_rin_d) * g.inv_dl_d;
    // azimuth
    const double num = X * dy - Y * dx, den = rho2 + rd;
    if (den > 0.0 && fabs(num) <= kSmall64 * den) {
      R.b2 += atan_small64(num * rcp64(den)) * g.inv_dph_d;
    } else {
      double ph = (nX * nX + nY * nY) > 0.0 ? atan2_64(nY, nX) : 0.0;
      if (ph < 0.0) ph += 6.283185307179586476925;
      R.b2 = ph * g.inv_dph_d;
    }
    if (R.b2 < 0.0) R.b2 += double(g.n2);
    if (R.b2 >= double(g.n2)) R.b2 -= double(g.n2);
    // colatitude
    const double e = 2.0 * rd + dd;
    const double rhoq = sqrt64(rho2 + e);
    const double dsum = rhoq + rho;
    const double drho = dsum > 0.0 ? e * rcp64(dsum) : 0.0;
    const double numt = Z * drho - rho * dz, dent = Z * nZ + rho * rhoq;
    if (dent > 0.0 && fabs(numt) <= kSmall64 * dent) R.b1 += atan_small64(numt * rcp64(dent)) * g.inv_dth_d;
    else R.b1 = atan2_64(rhoq, nZ) * g.inv_dth_d - 0.5;
  } else {
    R.b0 += dx * g.inv_sp_d[0];
    R.b1 += dy * g.inv_sp_d[1];
    R.b2 += dz * g.inv_sp_d[2];
  }
}

// FP32 index: add an increment to (cell, fraction) and bring the fraction back
// to [0, 1).
__device__ __forceinline__ void advance_cell(int& i, float& f, float d) {
  float x = f + d;
  float k = floorf(x);
  if (!(k >= -1.0e9f && k <= 1.0e9f)) k = 0.0f;  // NaN guard (the step is then non-finite)
  f = x - k;
  i += int(k);
}

// The same advance for FP32 state, all in FP32: the increments of (ln r, theta,
// phi) from r_i to r_i + d by the small-offset formulas of `locate` (they hold
// for any increment: log1p and the signed angles fall back to their general
// forms), the periodic axis wrapped back into [0, n2).
template <int KIND, class Real>
__device__ __forceinline__ void index_advance(const DevGeom& g, RayStateT<float, Real>& R, float dx, float dy,
                                              float dz) {
  float d0, d1, d2;
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    const float X = R.rx, Y = R.ry, Z = R.rz;  // old origin
    const float rho2 = X * X + Y * Y, r2 = rho2 + Z * Z, rho = sqrt_r(rho2);
    const float rd = X * dx + Y * dy;
    const float dd = dx * dx + dy * dy;
    const float c = 2.0f * (rd + Z * dz) + (dd + dz * dz);
    d0 = 0.5f * log1p_inc(c * rcpf(r2)) * g.inv_dl;
    d2 = atan2_inc(X * dy - Y * dx, rho2 + rd) * g.inv_dph;
    const float e = 2.0f * rd + dd;
    const float rhoq = sqrt_r(fmaxf(rho2 + e, 0.0f));
    const float dsum = rhoq + rho;
    const float drho = dsum > 0.0f ? e * rcpf(dsum) : 0.0f;
    d1 = atan2_inc(Z * drho - rho * dz, Z * (Z + dz) + rho * rhoq) * g.inv_dth;
  } else {
    d0 = dx * g.inv_sp[0];
    d1 = dy * g.inv_sp[1];
    d2 = dz * g.inv_sp[2];
  }
  advance_cell(R.i0, R.fr0, d0);
  advance_cell(R.i1, R.fr1, d1);
  advance_cell(R.i2, R.fr2, d2);
  if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
    if (R.i2 >= g.n2) R.i2 -= g.n2;
    else if (R.i2 < 0) R.i2 += g.n2;
  }
}

// Launch (Sec. 3.2): pixel centre (pu, pv) on the image plane; the ray starts on
// the r_max sphere and travels along -o.
__device__ __forceinline__ void pixel_start(const TraceArgs& a, int i, int j, double& pu, double& pv, double& b2,
                                            double& x0) {
  pu = -a.half_u + (j + 0.5) * 2.0 * a.half_u / a.nu;
  pv = -a.half_v + (i + 0.5) * 2.0 * a.half_v / a.nv;
  b2 = pu * pu + pv * pv;
  const double rmax = a.g.r_max;
  x0 = (b2 < rmax * rmax) ? sqrt(rmax * rmax - b2) : 0.0;
}

// Start ray `pix` (flat pixel index) of image `img` (= model * n_freq + freq):
// r0 and its grid index come from the per-pixel table, p0 = n(r0) (-o).
// Returns false for a ray that misses the model (its output is written).
template <class S, class Real>
__device__ __forceinline__ bool init_ray(const TraceArgs& a, int img, int pix, RayStateT<S, Real>& R, CellCache& C) {
  const int npx = a.nu * a.nv;
  const int model = img / a.n_freq;
  const int fi = img - model * a.n_freq;
  const int id = img * npx + pix;
  const double* L = a.launch + size_t(pix) * 6;
  if (L[3] < 0.0) {  // missing pixel: L[0..2] is its image-plane point, L[4] its impact parameter
    write_miss(a, id, L[4], L[0], L[1], L[2]);
    return false;
  }
  R.rx = S(L[0]); R.ry = S(L[1]); R.rz = S(L[2]);
  if constexpr (std::is_same<S, double>::value) {
    R.b0 = L[3]; R.b1 = L[4]; R.b2 = L[5];
  } else {
    split_index(L[3], R.i0, R.fr0);
    split_index(L[4], R.i1, R.fr1);
    split_index(L[5], R.i2, R.fr2);
  }
  C.key = -1;  // the lane's cached cell may belong to another model
  const double xf = a.xf[fi];
  R.xff = float(xf);
  R.cf = float(-0.5 * xf);
  R.cfd = -0.5 * xf;
  R.f2 = float(a.freqs[fi] * a.freqs[fi]);
  R.lnf = a.lnf[fi];
  R.nfg = a.models[model].nfg;
  R.te = a.models[model].te;
  R.id = id;
  double nidx = 1.0;
  if (a.flags & RT_USE_REFRACTION) {
    const float n2 = 1.0f - R.xff * a.launch_ne[size_t(model) * npx + pix];
    nidx = n2 > 0.f ? double(sqrt_fast(n2)) : 0.0;
  }
  R.px = S(-nidx * a.o[0]); R.py = S(-nidx * a.o[1]); R.pz = S(-nidx * a.o[2]);
  R.A = Real(0); R.lam_tot = Real(0); R.tau = Real(0); R.lns = Real(0); R.s_arc = S(0);
  R.rmin = float(a.g.r_max);
  R.lam_end = 1.0f;
  R.n = 0;
  R.code = kRunning;
  R.path_slot = (a.n_path > 0) ? find_path_slot(a, id) : -1;
  R.path_len = 0;
  return true;
}

// Carried tube at the launch: neighbours eps = eta ds_max away across the launch
// direction d = -o (the Eq. 6 basis of d), each with the wavevector n(start) d;
// ln S at the start point.
template <int KIND>
__device__ __forceinline__ void init_tube(const TraceArgs& a, RayState& R, CellCache& C) {
  const double dx = -a.o[0], dy = -a.o[1], dz = -a.o[2];
  double c1x, c1y, c1z;
  if (fabs(dz) > 0.9) { c1x = dz; c1y = 0.0; c1z = -dx; }   // y x d
  else { c1x = -dy; c1y = dx; c1z = 0.0; }                  // z x d
  const double ci = rsqrt64(c1x * c1x + c1y * c1y + c1z * c1z);
  const double e[2][3] = {{c1x * ci, c1y * ci, c1z * ci},
                          {dy * c1z * ci - dz * c1y * ci, dz * c1x * ci - dx * c1z * ci, dx * c1y * ci - dy * c1x * ci}};
  const double eps = a.ds_max_d * double(a.eta);
  StepOrigin O;
  make_origin<KIND>(R, O);
  // the wavevector difference (n_j - n_0) d from the difference of n_e, so that
  // it is not lost in the rounding of n (n_j - n_0 = -Xf (ne_j - ne_0) / (n_j + n_0))
  float ne0, te0;
  eval_value<KIND, true>(a.g, R.nfg, R.te, C, O, 0.f, 0.f, 0.f, ne0, te0);
  const double xf = -2.0 * R.cfd;
  const double n0 = sqrt64(fmax(1.0 - xf * double(ne0), 0.0));
  for (int j = 0; j < 2; ++j) {
    float ne, te;
    eval_value<KIND>(a.g, R.nfg, R.te, C, O, float(eps * e[j][0]), float(eps * e[j][1]), float(eps * e[j][2]), ne, te);
    const double nj = sqrt64(fmax(1.0 - xf * double(ne), 0.0));
    const double dn = (nj + n0) > 0.0 ? -xf * (double(ne) - double(ne0)) * rcp64(nj + n0) : 0.0;
    for (int k = 0; k < 3; ++k) {
      R.nb_r[j][k] = eps * e[j][k];
      R.nb_p[j][k] = dn * (k == 0 ? dx : k == 1 ? dy : dz);
    }
  }
  // S_0 = |(eps e1 x eps e2) . d| = eps^2
  R.tube_ln_s = log(eps * eps);
}

template <class S, class Real>
__device__ __forceinline__ void finish_ray(const TraceArgs& a, const RayStateT<S, Real>& R) {
  const double tbc = (R.code == kHit) ? a.tb_inner : a.tb_sky;
  const float trans = __builtin_amdgcn_exp2f(-1.44269504089f * float(R.lam_tot));
  a.tb[R.id] = float(double(R.A) + double(trans) * tbc);
  if (a.info) {
    rt_ray_info inf;
    inf.n_steps = R.n;
    inf.code = int8_t(R.code);
    inf.flags = ((R.code == kExit || R.code == kHit) && (R.lam_end < 1e-4f || R.lam_end > 1.0f - 1e-4f))
                    ? int8_t(RT_RAY_FLAG_MARGINAL) : int8_t(0);
    inf._pad[0] = inf._pad[1] = 0;
    inf.exit_pos[0] = float(R.rx); inf.exit_pos[1] = float(R.ry); inf.exit_pos[2] = float(R.rz);
    inf.tau = float(R.tau);
    inf.ln_s_end = float(R.lns);
    inf.r_min = fminf(R.rmin, sqrt_fast(float(R.rx * R.rx + R.ry * R.ry + R.rz * R.rz)));
    a.info[R.id] = inf;
  }
  if (R.path_slot >= 0) a.path_len[R.path_slot] = R.path_len;
}

// Segment factor of the exact transfer update over one segment, in FP32:
// phi = (1 - e^{-x}) / x (series below |x| = 1/16).
__device__ __forceinline__ float segment_phi(float x) {
  if (fabsf(x) <= 0.0625f) {
    float s = 1.0f / 720.0f;
    s = fmaf(s, -x, 1.0f / 120.0f);
    s = fmaf(s, -x, 1.0f / 24.0f);
    s = fmaf(s, -x, 1.0f / 6.0f);
    s = fmaf(s, -x, 0.5f);
    return fmaf(s, -x, 1.0f);
  }
  return (1.0f - __builtin_amdgcn_exp2f(-1.44269504089f * x)) * rcpf(x);
}

// Tracing mode of ray_step: from the call's flags, or fixed at compile time.
enum : int { kModeFlags = 0, kModeLos = 1, kModeNoMag = 2, kModeFull = 3, kModeCarried = 4 };

// One central RK4 step with its two perturbed retraces, termination test and
// transfer segment.  Returns the termination code (kRunning to continue); on
// termination R holds the end point, the code and the last-step fraction.
// TAPE: when tp is not null, also write the step's record (fields kTape*,
// field f at tp[f * ts]).
// S, the precision of the state and of the step increments, comes from the ray
// state's type; Real, that of the ray-tube area and the transfer, from MIXED.
template <bool MIXED, int KIND, int MODE = kModeFlags, bool TAPE = false, class S>
__device__ __forceinline__ int ray_step(const TraceArgs& a, RayStateT<S, typename RealOf<MIXED>::T>& R, CellCache& C,
                                         float* tp = nullptr, size_t ts = 0) {
  using Real = typename RealOf<MIXED>::T;
  constexpr bool s64 = std::is_same<S, double>::value;
  const bool refr = (MODE == kModeFlags) ? (a.flags & RT_USE_REFRACTION) != 0 : (MODE != kModeLos);
  const bool mag = (MODE == kModeFlags) ? refr && (a.flags & RT_USE_MAGNIFICATION) != 0 : (MODE == kModeFull);
  constexpr bool carried = MODE == kModeCarried;
  static_assert(s64 || (!carried && !TAPE), "carried tubes and the adjoint record use FP64 state");

  // All evaluation points of this step are r_i + (FP32 offset).
  StepOrigin O;
  make_origin<KIND>(R, O);
  const float pxf = float(R.px), pyf = float(R.py), pzf = float(R.pz);
  float h;
  S hd;
  S drx, dry, drz, dpx = S(0), dpy = S(0), dpz = S(0);
  float d2x = 0.f, d2y = 0.f, d2z = 0.f, d3x = 0.f, d3y = 0.f, d3z = 0.f;
  float F1x = 0.f, F1y = 0.f, F1z = 0.f, F2x = 0.f, F2y = 0.f, F2z = 0.f, F3x = 0.f, F3y = 0.f, F3z = 0.f;
  float sx = 0.f, sy = 0.f, sz = 0.f;                 // g1 + g2 + g3
  float tx = 0.f, ty = 0.f, tz = 0.f;                 // g1 + 2 g2 + 2 g3 + g4
  if (refr) {
    // Stage 1 at r_i also sets the step: dt = ds_max / max(n(r_i), n_floor).
    float ne, gx, gy, gz;
    eval_grad<KIND, true>(a.g, R.nfg, R.te, C, O, 0.f, 0.f, 0.f, ne, gx, gy, gz);
    F1x = R.cf * gx; F1y = R.cf * gy; F1z = R.cf * gz;
    sx = gx; sy = gy; sz = gz;
    tx = gx; ty = gy; tz = gz;
    const float n2 = 1.0f - R.xff * ne;
    const float ni = n2 > 0.f ? sqrt_fast(n2) : 0.f;
    if (TAPE && tp) {
      tp[kTapeNi * ts] = ni;
      tp[kTapeF1 * ts] = F1x; tp[(kTapeF1 + 1) * ts] = F1y; tp[(kTapeF1 + 2) * ts] = F1z;
    }
    if constexpr (s64) hd = (ni > a.n_floor) ? a.ds_max_d * rcp64(double(ni)) : a.ds_max_d * rcp64(a.n_floor_d);
    else hd = a.ds_max * rcpf(fmaxf(ni, a.n_floor));
    h = float(hd);
    const float hh = 0.5f * h;
    d2x = hh * pxf; d2y = hh * pyf; d2z = hh * pzf;
    eval_grad<KIND>(a.g, R.nfg, R.te, C, O, d2x, d2y, d2z, ne, gx, gy, gz);
    F2x = R.cf * gx; F2y = R.cf * gy; F2z = R.cf * gz;
    if (TAPE && tp) { tp[kTapeF2 * ts] = F2x; tp[(kTapeF2 + 1) * ts] = F2y; tp[(kTapeF2 + 2) * ts] = F2z; }
    sx += gx; sy += gy; sz += gz;
    tx = fmaf(2.f, gx, tx); ty = fmaf(2.f, gy, ty); tz = fmaf(2.f, gz, tz);
    d3x = hh * (pxf + hh * F1x); d3y = hh * (pyf + hh * F1y); d3z = hh * (pzf + hh * F1z);
    eval_grad<KIND>(a.g, R.nfg, R.te, C, O, d3x, d3y, d3z, ne, gx, gy, gz);
    F3x = R.cf * gx; F3y = R.cf * gy; F3z = R.cf * gz;
    sx += gx; sy += gy; sz += gz;
    tx = fmaf(2.f, gx, tx); ty = fmaf(2.f, gy, ty); tz = fmaf(2.f, gz, tz);
    eval_grad<KIND>(a.g, R.nfg, R.te, C, O, h * (pxf + hh * F2x), h * (pyf + hh * F2y), h * (pzf + hh * F2z), ne, gx,
                    gy, gz);
    tx += gx; ty += gy; tz += gz;
    if (TAPE && tp) {
      tp[kTapeS * ts] = sx; tp[(kTapeS + 1) * ts] = sy; tp[(kTapeS + 2) * ts] = sz;
      tp[kTapeT * ts] = tx; tp[(kTapeT + 1) * ts] = ty; tp[(kTapeT + 2) * ts] = tz;
    }
    // RK4: dr = h p + h^2/6 (F1 + F2 + F3), dp = h/6 (F1 + 2 F2 + 2 F3 + F4),
    // F = -1/2 Xf grad n_e, the coefficient applied in the state's precision.
    const S c6 = (s64 ? S(R.cfd) : S(R.cf)) * hd * S(1.0 / 6.0);
    drx = hd * R.px + hd * c6 * S(sx);
    dry = hd * R.py + hd * c6 * S(sy);
    drz = hd * R.pz + hd * c6 * S(sz);
    dpx = c6 * S(tx);
    dpy = c6 * S(ty);
    dpz = c6 * S(tz);
  } else {
    // Straight line of sight: no force, |p| = 1, dt = ds_max.
    h = a.ds_max;
    hd = s64 ? S(a.ds_max_d) : S(a.ds_max);
    drx = hd * R.px; dry = hd * R.py; drz = hd * R.pz;
  }
  if constexpr (carried) {
    // The two neighbour rays take the same RK4 step from r_i + dr_j with wavevector
    // p_i + dp_j; their stages are evaluated at FP32 offsets from r_i, and their
    // separations advance by the differences of the increments (FP64):
    // d(dr_j) = h dp_j + h^2/6 cf (s_j - s), d(dp_j) = h/6 cf (t_j - t).
    const float hh = 0.5f * h;
    const double c6 = R.cfd * hd * (1.0 / 6.0);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double qx = R.px + R.nb_p[j][0], qy = R.py + R.nb_p[j][1], qz = R.pz + R.nb_p[j][2];
      const float bx = float(R.nb_r[j][0]), by = float(R.nb_r[j][1]), bz = float(R.nb_r[j][2]);
      const float qxf = float(qx), qyf = float(qy), qzf = float(qz);
      float ne, gx, gy, gz;
      eval_grad<KIND>(a.g, R.nfg, R.te, C, O, bx, by, bz, ne, gx, gy, gz);
      const float G1x = R.cf * gx, G1y = R.cf * gy, G1z = R.cf * gz;
      float sjx = gx, sjy = gy, sjz = gz, tjx = gx, tjy = gy, tjz = gz;
      eval_grad<KIND>(a.g, R.nfg, R.te, C, O, bx + hh * qxf, by + hh * qyf, bz + hh * qzf, ne, gx, gy, gz);
      const float G2x = R.cf * gx, G2y = R.cf * gy, G2z = R.cf * gz;
      sjx += gx; sjy += gy; sjz += gz;
      tjx = fmaf(2.f, gx, tjx); tjy = fmaf(2.f, gy, tjy); tjz = fmaf(2.f, gz, tjz);
      eval_grad<KIND>(a.g, R.nfg, R.te, C, O, bx + hh * (qxf + hh * G1x), by + hh * (qyf + hh * G1y),
                      bz + hh * (qzf + hh * G1z), ne, gx, gy, gz);
      sjx += gx; sjy += gy; sjz += gz;
      tjx = fmaf(2.f, gx, tjx); tjy = fmaf(2.f, gy, tjy); tjz = fmaf(2.f, gz, tjz);
      eval_grad<KIND>(a.g, R.nfg, R.te, C, O, bx + h * (qxf + hh * G2x), by + h * (qyf + hh * G2y),
                      bz + h * (qzf + hh * G2z), ne, gx, gy, gz);
      tjx += gx; tjy += gy; tjz += gz;
      R.nb_r[j][0] += hd * R.nb_p[j][0] + hd * c6 * double(sjx - sx);
      R.nb_r[j][1] += hd * R.nb_p[j][1] + hd * c6 * double(sjy - sy);
      R.nb_r[j][2] += hd * R.nb_p[j][2] + hd * c6 * double(sjz - sz);
      R.nb_p[j][0] += c6 * double(tjx - tx);
      R.nb_p[j][1] += c6 * double(tjy - ty);
      R.nb_p[j][2] += c6 * double(tjz - tz);
    }
  }
  R.n += 1;
  if (!(isfinite(drx) && isfinite(dry) && isfinite(drz) && isfinite(dpx) && isfinite(dpy) && isfinite(dpz))) {
    R.code = kNonfinite;
    R.lam_end = 1.0f;
    return kNonfinite;
  }
  R.px += dpx; R.py += dpy; R.pz += dpz;  // p is not used again in this step

  // Eq. 5: chord direction (the chord is exactly the increment dr).
  const Real dx = Real(drx), dy = Real(dry), dz = Real(drz);
  const Real ds2 = dx * dx + dy * dy + dz * dz;
  const Real inv_ds = rsqrt_r(ds2);
  const Real ds = ds2 * inv_ds;
  float lnM = 0.0f;
  if (mag) {
    const Real tx = dx * inv_ds, ty = dy * inv_ds, tz = dz * inv_ds;
    // Eq. 6: a = z unless |t_z| is near 1, then y; e1 = a x t / |a x t|, e2 = t x e1.
    Real c1x, c1y, c1z;
    if (fabs(tz) > Real(0.9)) { c1x = tz; c1y = Real(0); c1z = -tx; }
    else { c1x = -ty; c1y = tx; c1z = Real(0); }
    const Real ci = rsqrt_r(c1x * c1x + c1y * c1y + c1z * c1z);
    const Real e1x = c1x * ci, e1y = c1y * ci, e1z = c1z * ci;
    const Real eps = Real(a.eta) * ds;  // Eq. 8
    // Eqs. 7 and 9 in difference form: the perturbed ray starts at r_i + eps e_j with
    // the central wavevector; its RK4 end point minus the central one is
    // eps e_j + h^2/6 (dF1 + dF2 + dF3), dF_k the force differences at the first
    // three stages (the fourth stage only moves p, which is discarded).
    const float hh = 0.5f * h, hq = hh * hh, hh6 = h * h * (1.0f / 6.0f);
    Real s1x = 0, s1y = 0, s1z = 0, det = 0;
#pragma unroll 1
    for (int jj = 0; jj < 2; ++jj) {
      Real ex = e1x, ey = e1y, ez = e1z;
      if (jj == 1) { ex = ty * e1z - tz * e1y; ey = tz * e1x - tx * e1z; ez = tx * e1y - ty * e1x; }
      const Real d0x = eps * ex, d0y = eps * ey, d0z = eps * ez;
      const float fx = float(d0x), fy = float(d0y), fz = float(d0z);
      float ne, gx, gy, gz;
      eval_grad<KIND>(a.g, R.nfg, R.te, C, O, fx, fy, fz, ne, gx, gy, gz);
      const float q1x = R.cf * gx - F1x, q1y = R.cf * gy - F1y, q1z = R.cf * gz - F1z;
      eval_grad<KIND>(a.g, R.nfg, R.te, C, O, d2x + fx, d2y + fy, d2z + fz, ne, gx, gy, gz);
      float ax = q1x + (R.cf * gx - F2x), ay = q1y + (R.cf * gy - F2y), az = q1z + (R.cf * gz - F2z);
      eval_grad<KIND>(a.g, R.nfg, R.te, C, O, d3x + fx + hq * q1x, d3y + fy + hq * q1y, d3z + fz + hq * q1z, ne, gx,
                      gy, gz);
      ax += R.cf * gx - F3x; ay += R.cf * gy - F3y; az += R.cf * gz - F3z;
      if (TAPE && tp) {
        float* q = tp + size_t(kTapeQ + 3 * jj) * ts;
        q[0] = q1x; q[ts] = q1y; q[2 * ts] = q1z;
        float* f = tp + size_t(kTapeA + 3 * jj) * ts;
        f[0] = ax; f[ts] = ay; f[2 * ts] = az;
      }
      const Real sx = d0x + Real(hh6 * ax), sy = d0y + Real(hh6 * ay), sz = d0z + Real(hh6 * az);
      if (jj == 0) { s1x = sx; s1y = sy; s1z = sz; }
      else det = (s1y * sz - s1z * sy) * tx + (s1z * sx - s1x * sz) * ty + (s1x * sy - s1y * sx) * tz;
    }
    // Eqs. 10-11: M = |(dr1 x dr2) . t| / eps^2; ln M from the accurately formed M - 1.
    const Real mm1 = fabs(det) * rcp_r(eps * eps) - Real(1);
    lnM = fast_log1pf(float(mm1));
  }
  if constexpr (carried) {
    // cross-section of the carried tube at r_{i+1}: |(dr_a x dr_b) . p_hat|
    const double* ua = R.nb_r[0];
    const double* ub = R.nb_r[1];
    const double cx = ua[1] * ub[2] - ua[2] * ub[1], cy = ua[2] * ub[0] - ua[0] * ub[2], cz = ua[0] * ub[1] - ua[1] * ub[0];
    const double pp = R.px * R.px + R.py * R.py + R.pz * R.pz;
    const double area = fabs(cx * R.px + cy * R.py + cz * R.pz) * rsqrt64(pp);
    const double ln_s = log(area);
    lnM = float(ln_s - R.tube_ln_s);
    R.tube_ln_s = ln_s;
  }

  // Termination on the two spheres, last chord truncated at the crossing.
  const S nx = R.rx + drx, ny = R.ry + dry, nz = R.rz + drz;
  const S r1sq = nx * nx + ny * ny + nz * nz;
  int code = kRunning;
  S lam = S(1);
  if (a.g.has_inner && r1sq <= S(a.g.r_in * a.g.r_in)) {
    code = kHit;
    lam = crossing<S>(R.rx, R.ry, R.rz, drx, dry, drz, a.g.r_in, false);
  } else if (r1sq >= S(a.g.r_max * a.g.r_max) && R.n >= 2) {
    code = kExit;
    lam = crossing<S>(R.rx, R.ry, R.rz, drx, dry, drz, a.g.r_max, true);
  } else if (R.n == a.max_steps) {
    code = kMaxSteps;
  }

  // Segment at the chord midpoint: free-free kappa*n, dtau = kappa*n R_sun lam dt,
  // gamma = -lam ln M (the d ln S/ds term over the segment, in the transfer direction).
  const float hl = 0.5f * float(lam);
  float ne_m, te_m;
  eval_value<KIND>(a.g, R.nfg, R.te, C, O, hl * float(drx), hl * float(dry), hl * float(drz), ne_m, te_m);
  if (TAPE && tp) { tp[kTapeNeM * ts] = ne_m; tp[kTapeTeM * ts] = te_m; }
  Real dtau = Real(0);
  if (!(a.flags & RT_TEST_NO_ABSORPTION)) {
    const float lt = __builtin_amdgcn_logf(te_m) * 0.69314718056f;
    const float lnl = (te_m >= 2.0e5f) ? 24.5f + lt - R.lnf : 18.2f + 1.5f * lt - R.lnf;
    const float kn = kFFCoefF * ne_m * ne_m * lnl * rcpf(R.f2 * te_m * sqrt_fast(te_m));
    dtau = Real(kn) * (Real(kRsunCm) * Real(lam) * Real(hd));
  }
  const Real gamma = -Real(lam) * Real(lnM);
  const Real xs = dtau + gamma;
  // front to back: A += e^{-Lambda} T dtau phi(x), Lambda += x; the transmittance
  // is formed from the accumulated Lambda each step, so its error does not compound
  const float trans = __builtin_amdgcn_exp2f(-1.44269504089f * float(R.lam_tot));
  R.A = R.A + Real(trans) * (Real(te_m) * dtau * Real(segment_phi(float(xs))));
  R.lam_tot = R.lam_tot + xs;
  R.tau = R.tau + dtau;
  R.lns = R.lns + Real(lam) * Real(lnM);

  if (R.path_slot >= 0) {
    R.s_arc += lam * S(ds);
    if (R.path_len < a.path_cap) {
      float* rec = a.path_out + (size_t(R.path_slot) * a.path_cap + R.path_len) * kPathStride;
      rec[0] = float(R.rx + lam * drx); rec[1] = float(R.ry + lam * dry); rec[2] = float(R.rz + lam * drz);
      rec[3] = float(R.s_arc); rec[4] = lnM; rec[5] = lnM / float(ds);
      rec[6] = float(R.tau); rec[7] = ne_m; rec[8] = te_m;
      R.path_len += 1;
    }
  }

  if (code != kRunning) {
    R.rx += lam * drx; R.ry += lam * dry; R.rz += lam * drz;
    R.code = code;
    R.lam_end = float(lam);
    return code;
  }
  index_advance<KIND>(a.g, R, drx, dry, drz);
  R.rx = nx; R.ry = ny; R.rz = nz;
  R.rmin = fminf(R.rmin, sqrt_fast(float(r1sq)));
  return kRunning;
}

}  // namespace rt
