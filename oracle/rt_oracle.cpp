// FP64 CPU oracle for refractive radio ray tracing with step-wise ray-tube
// magnification and thermal free-free transfer.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
// reference that the GPU library is checked against.  Only the tests, the
// smoke check and the benchmark's CPU-baseline leg load it.  It shares no code,
// header, table or helper with the GPU library.
//
// What it follows (paper: "Modeling the Thermal Low-Frequency Radio Sun with
// Ray Tracing"):
//   * Hamiltonian ray equations (Sec. 2.1, Eq. 4) with the cold-plasma index
//     n^2 = 1 - f_p^2/f^2, f_p = 8.98 kHz sqrt(n_e), written for the normalised
//     wavevector p = c k / omega:  dr/dt = p,  dp/dt = -1/2 grad X,
//     X = (8.98e3)^2 n_e / f^2, so |p| = n and ds = n dt.  Classical RK4.
//   * Step-wise perturbation retracing (Sec. 2.1, Eqs. 5-11): chord direction,
//     reference axis, transverse basis, perturbed starts at eps = eta*|chord|,
//     one RK4 step with the central wavevector, separations, area, magnification.
//     The factor 1/2 of the area estimate is dropped (parallelogram area), so an
//     undeformed tube gives M = 1 as the text around Eq. 11 requires.
//   * Transfer with the geometric term (Eqs. 2-3, 12), solved from the far end
//     of each ray back toward the observer after tracing has finished (Sec. 3.2).
//     Per segment the exact solution for constant kappa, T and d ln S/ds is used.
//   * Thermal free-free absorption in its Rayleigh-Jeans closed form with the
//     two-branch Coulomb logarithm (Dulk 1985, ARA&A 23, 169, cited in Sec. 1).
//   * Optionally (carried_tube) the tube cross-section S of Eqs. 2-3 from two
//     neighbour rays launched once across the initial direction and stepped
//     beside the ray for its whole length, ln M of a step = ln(S_{i+1}/S_i);
//     each ray also reports the smallest ln(S/S_0) over its step points.
//
// A second stepper (Dormand-Prince 5(4) with error control) traces the central
// ray only; it is the physics reference for invariants, not for parity.
//
// Parity-unpinned parts are listed in the tests' docstrings.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <type_traits>
#include <vector>

namespace orc {

constexpr double kPi = 3.14159265358979323846;
constexpr double kRsunCm = 6.957e10;   // nominal solar radius [cm]
constexpr double kFpCoef = 8.98e3;     // f_p [Hz] = 8.98e3 sqrt(n_e [cm^-3])
constexpr double kFFCoef = 9.78e-3;    // free-free absorption constant (Dulk 1985)

enum Code : int32_t { RUNNING = 0, EXIT_OUTER = 1, HIT_INNER = 2, MISS = 3, MAX_STEPS = 4, NONFINITE = 5 };
enum Flag : int32_t { GRAZING = 1, MARGINAL = 2, POLAR = 4 };

enum MediumKind : int32_t {
  GRID_SPHERICAL_LOGR = 0, GRID_CARTESIAN = 1,
  ANALYTIC_BA = 10, ANALYTIC_UNIFORM = 11, ANALYTIC_SLAB = 12, ANALYTIC_LENS = 13
};

// ---------------------------------------------------------------------------
// Forward-mode dual number (value + one directional derivative).
// ---------------------------------------------------------------------------
struct Dual {
  double v = 0, d = 0;
  Dual() = default;
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return {s, a.d / (2.0 * s)}; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return {e, a.d * e}; }
inline Dual expm1(Dual a) { return {std::expm1(a.v), a.d * std::exp(a.v)}; }
inline Dual log(Dual a) { return {std::log(a.v), a.d / a.v}; }
inline Dual pow(Dual a, double k) { return {std::pow(a.v, k), a.d * k * std::pow(a.v, k - 1.0)}; }
inline Dual atan2(Dual y, Dual x) {
  double r2 = x.v * x.v + y.v * y.v;
  return {std::atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2};
}
inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline bool finite_s(double x) { return std::isfinite(x); }
inline bool finite_s(const Dual& x) { return std::isfinite(x.v); }

// ---------------------------------------------------------------------------
// Reverse-mode scalar on a per-thread tape.  Every operation whose operands are
// not all constants appends one node (up to two parents and the local partial
// derivatives); a model value read from the grid appends a leaf node that names
// its vertex and whether it is n_e or T, with the partial d value / d ln value.
// One ray is recorded, swept backward from its output, then the tape is reset.
// ---------------------------------------------------------------------------
constexpr int32_t kNoParent = -1, kLeafNe = -2, kLeafTe = -3;
struct TapeNode {
  int32_t a, b;      // parents (node indices), or kNoParent; a leaf has a = kLeafNe / kLeafTe, b = vertex
  double da, db;     // partial derivatives w.r.t. a and b
};
struct Tape {
  std::vector<TapeNode> nodes;
};
inline Tape*& tape_ref() {
  static thread_local Tape* t = nullptr;
  return t;
}
struct Rev {
  double v = 0;
  int32_t i = kNoParent;  // node index; kNoParent for a constant
  Rev() = default;
  Rev(double x) : v(x), i(kNoParent) {}
};
inline Rev rev_node(double v, int32_t a, double da, int32_t b, double db) {
  if (a == kNoParent && b == kNoParent) return Rev(v);
  Tape* t = tape_ref();
  if (a == kNoParent) { a = b; da = db; b = kNoParent; db = 0.0; }
  t->nodes.push_back({a, b, da, db});
  Rev r(v);
  r.i = int32_t(t->nodes.size() - 1);
  return r;
}
inline Rev rev_leaf(double v, int32_t kind, size_t vertex) {
  Tape* t = tape_ref();
  t->nodes.push_back({kind, int32_t(vertex), v, 0.0});
  Rev r(v);
  r.i = int32_t(t->nodes.size() - 1);
  return r;
}
inline Rev operator+(Rev a, Rev b) { return rev_node(a.v + b.v, a.i, 1.0, b.i, 1.0); }
inline Rev operator-(Rev a, Rev b) { return rev_node(a.v - b.v, a.i, 1.0, b.i, -1.0); }
inline Rev operator-(Rev a) { return rev_node(-a.v, a.i, -1.0, kNoParent, 0.0); }
inline Rev operator*(Rev a, Rev b) { return rev_node(a.v * b.v, a.i, b.v, b.i, a.v); }
inline Rev operator/(Rev a, Rev b) { return rev_node(a.v / b.v, a.i, 1.0 / b.v, b.i, -a.v / (b.v * b.v)); }
inline Rev sqrt(Rev a) { double s = std::sqrt(a.v); return rev_node(s, a.i, 0.5 / s, kNoParent, 0.0); }
inline Rev exp(Rev a) { double e = std::exp(a.v); return rev_node(e, a.i, e, kNoParent, 0.0); }
inline Rev expm1(Rev a) { return rev_node(std::expm1(a.v), a.i, std::exp(a.v), kNoParent, 0.0); }
inline Rev log(Rev a) { return rev_node(std::log(a.v), a.i, 1.0 / a.v, kNoParent, 0.0); }
inline Rev pow(Rev a, double k) { return rev_node(std::pow(a.v, k), a.i, k * std::pow(a.v, k - 1.0), kNoParent, 0.0); }
inline Rev atan2(Rev y, Rev x) {
  double r2 = x.v * x.v + y.v * y.v;
  return rev_node(std::atan2(y.v, x.v), y.i, x.v / r2, x.i, -y.v / r2);
}
inline Rev fabs(Rev a) { return a.v < 0 ? -a : a; }
inline double val(const Rev& x) { return x.v; }
inline bool finite_s(const Rev& x) { return std::isfinite(x.v); }

// Backward sweep of the current tape from node `out` with seed `w`; leaf
// adjoints (already d/d ln) are added to gne / gte.
inline void rev_sweep(const Rev& out, double w, double* gne, double* gte, std::vector<double>& adj) {
  Tape* t = tape_ref();
  if (out.i == kNoParent) return;
  adj.assign(size_t(out.i) + 1, 0.0);
  adj[size_t(out.i)] = w;
  for (int64_t k = out.i; k >= 0; --k) {
    const double g = adj[size_t(k)];
    if (g == 0.0) continue;
    const TapeNode& nd = t->nodes[size_t(k)];
    if (nd.a == kLeafNe) { gne[nd.b] += g * nd.da; continue; }
    if (nd.a == kLeafTe) { gte[nd.b] += g * nd.da; continue; }
    if (nd.a >= 0) adj[size_t(nd.a)] += g * nd.da;
    if (nd.b >= 0) adj[size_t(nd.b)] += g * nd.db;
  }
}

// ---------------------------------------------------------------------------
// Small vector helpers.
// ---------------------------------------------------------------------------
template <class S> struct V3 { S x, y, z; };
template <class S> V3<S> operator+(const V3<S>& a, const V3<S>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> V3<S> operator-(const V3<S>& a, const V3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S, class T> V3<S> operator*(const T& s, const V3<S>& a) { return {S(s) * a.x, S(s) * a.y, S(s) * a.z}; }
template <class S> S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class S> S norm(const V3<S>& a) { using std::sqrt; return sqrt(dot(a, a)); }
template <class S> V3<S> lift(const V3<double>& a) { return {S(a.x), S(a.y), S(a.z)}; }

// ---------------------------------------------------------------------------
// Medium description (shared layout with the Python wrapper).
// ---------------------------------------------------------------------------
struct Medium {
  int32_t kind;
  int32_t n0, n1, n2;          // grid sizes: (N_r, N_theta, N_phi) or (N_x, N_y, N_z)
  double r_in, r_max;          // termination spheres [R_sun]; r_in <= 0 disables the inner one
  double origin[3], spacing[3];// Cartesian grid
  const float* ne;             // grid values, C-order [n0][n1][n2]
  const float* te;
  double a0, a1, a2;           // analytic parameters
  double t_const;              // temperature of analytic media [K]
};

struct Params {
  int32_t stepper;             // 0 = RK4 mirror, 1 = Dormand-Prince 5(4)
  int32_t use_refraction;
  int32_t use_magnification;
  int32_t no_absorption;
  double ds_max, n_floor;
  int32_t max_steps;
  int32_t twin_check;
  double eta;                  // perturb_ratio
  double tb_inner, tb_sky;
  double dp_rtol, dp_atol;
  int32_t carried_tube;        // 1: tube area from two neighbour rays carried along the whole ray
  int32_t _pad;
  double twin_exit_tol;        // twin check: exit movement [R_sun] that marks a ray ill-conditioned
};

struct Image {
  double obs_dir[3];
  double up[3];
  int32_t nu, nv;
  double half_u, half_v;
};

struct Result {
  double tb, tau, ln_s_end, r_min;
  double exit_pos[3];
  double lam_last;
  double bouguer_drift;        // max |(|r x p| - L0)| / L0 over accepted steps
  double ham_drift;            // max abs(|p|^2 + X - 1) over accepted steps
  double ln_s_min;             // smallest ln(S/S_0) over the step points (0 at the start)
  double twin_dexit;           // exit movement of the twin ray [R_sun]; -1 if no twin was traced, +inf if its code differs
  int32_t n_steps, code, flags, _pad;
  uint64_t event_hash;         // hash of the ray's discrete decisions (orc_trace_pixels; 0 elsewhere)
};

constexpr int kPathStride = 12;  // x y z s lnM dlnS/ds tau_cum ne_m te_m dtau gamma dt

// Where corner values come from: plain reads for double; for AD scalars a
// source may attach derivatives to them.
struct PlainSource {
  const Medium* m;
  template <class S> S ne(size_t i) const { return S(double(m->ne[i])); }
  template <class S> S te(size_t i) const { return S(double(m->te[i])); }
};

// Directional derivative of everything w.r.t. (ln n_e, ln T) along (vn, vt).
struct DualSource {
  const Medium* m;
  const double* vn;  // per-vertex direction for ln n_e (or null)
  const double* vt;  // per-vertex direction for ln T (or null)
  template <class S> S ne(size_t i) const {
    double x = m->ne[i];
    return S(x, vn ? x * vn[i] : 0.0);
  }
  template <class S> S te(size_t i) const {
    double x = m->te[i];
    return S(x, vt ? x * vt[i] : 0.0);
  }
};

// Model values as tape leaves (gradient w.r.t. ln n_e and ln T per vertex).
struct RevSource {
  const Medium* m;
  template <class S> S ne(size_t i) const { return rev_leaf(double(m->ne[i]), kLeafNe, i); }
  template <class S> S te(size_t i) const { return rev_leaf(double(m->te[i]), kLeafTe, i); }
};

template <class S> struct Sample {
  S ne;
  V3<S> grad;   // grad n_e [cm^-3 / R_sun]
  S te;
};

// Record of a ray's discrete decisions (a diagnostic; no arithmetic depends on
// it): while a ray is traced for orc_trace_pixels, every medium evaluation adds
// its cell and edge clamps, and every step its step-floor branch, the reference
// axis of the basis and the sign of the area's triple product, to a running
// FNV-1a hash.  Two traces with equal hashes took the same discrete path, so
// along a continuous change of the model between them the traced map is smooth.
inline uint64_t*& event_hash_ref() {
  static thread_local uint64_t* h = nullptr;
  return h;
}
inline void event_mix(uint64_t v) {
  uint64_t* h = event_hash_ref();
  if (!h) return;
  for (int k = 0; k < 8; ++k) {
    *h ^= (v >> (8 * k)) & 0xffu;
    *h *= 0x100000001b3ull;
  }
}

// Clamp a continuous index to [0, n-1]; report whether it was outside.
template <class S> S clamp_index(const S& xi, int n, bool& clamped) {
  clamped = false;
  if (val(xi) < 0.0) { clamped = true; return S(0.0); }
  if (val(xi) > double(n - 1)) { clamped = true; return S(double(n - 1)); }
  return xi;
}

// Trilinear value and index-space gradient over one cell given 8 corner values
// f[i][j][k] (i along axis 0, ...), fractional offsets (u, v, w).
template <class S> void trilinear(const S f[2][2][2], const S& u, const S& v, const S& w,
                                  S& value, S& du, S& dv, S& dw) {
  S one(1.0);
  S f00 = f[0][0][0] * (one - w) + f[0][0][1] * w;
  S f01 = f[0][1][0] * (one - w) + f[0][1][1] * w;
  S f10 = f[1][0][0] * (one - w) + f[1][0][1] * w;
  S f11 = f[1][1][0] * (one - w) + f[1][1][1] * w;
  S f0 = f00 * (one - v) + f01 * v;
  S f1 = f10 * (one - v) + f11 * v;
  value = f0 * (one - u) + f1 * u;
  du = f1 - f0;
  dv = (f01 - f00) * (one - u) + (f11 - f10) * u;
  S g0 = (f[0][0][1] - f[0][0][0]) * (one - v) + (f[0][1][1] - f[0][1][0]) * v;
  S g1 = (f[1][0][1] - f[1][0][0]) * (one - v) + (f[1][1][1] - f[1][1][0]) * v;
  dw = g0 * (one - u) + g1 * u;
}

// Medium evaluation: n_e, grad n_e and T at a position.
template <class S, class Src>
Sample<S> eval_medium(const Medium& m, const Src& src, const V3<S>& pos, bool want_te) {
  using std::atan2; using std::log; using std::sqrt; using std::pow; using std::floor;
  Sample<S> out{S(0.0), {S(0.0), S(0.0), S(0.0)}, S(0.0)};
  switch (m.kind) {
    case GRID_SPHERICAL_LOGR: {
      // Spherical grid (Sec. 3.1): vertices log-spaced in r between r_in and r_max,
      // cell-centred in theta, periodic in phi.  n_e and T are trilinear in the
      // continuous index (ln r, theta, phi), clamped at the r and theta edges.
      // The density gradient that drives the rays is the trilinear interpolant of
      // per-vertex central differences in index space (one-sided at the r and theta
      // edges, periodic in phi), mapped to Cartesian with the spherical unit
      // vectors; it is continuous across cell faces and across the clamped edges.
      const int nr = m.n0, nt = m.n1, np = m.n2;
      const double dl = std::log(m.r_max / m.r_in) / double(nr - 1);
      const double dth = kPi / double(nt);
      const double dph = 2.0 * kPi / double(np);
      S r = sqrt(dot(pos, pos));
      S rho = sqrt(pos.x * pos.x + pos.y * pos.y);
      S theta = atan2(rho, pos.z);
      bool on_axis = val(rho) < 1e-12;
      S phi(0.0);
      if (!on_axis) {
        phi = atan2(pos.y, pos.x);
        if (val(phi) < 0.0) phi = phi + S(2.0 * kPi);
      }
      bool cr, ct;
      S xr = clamp_index((log(r) - S(std::log(m.r_in))) / S(dl), nr, cr);
      S xt = clamp_index(theta / S(dth) - S(0.5), nt, ct);
      S xp = phi / S(dph);
      int a = std::min(int(std::floor(val(xr))), nr - 2);
      int b = std::min(int(std::floor(val(xt))), nt - 2);
      int c = int(std::floor(val(xp)));
      S u = xr - S(double(a)), v = xt - S(double(b)), w = xp - S(double(c));
      c = ((c % np) + np) % np;
      event_mix((uint64_t(uint32_t(a)) << 42) ^ (uint64_t(uint32_t(b)) << 21) ^ uint64_t(uint32_t(c)) ^
                (uint64_t(cr) << 61) ^ (uint64_t(ct) << 62) ^ (uint64_t(on_axis) << 63));
      auto at = [&](int i, int j, int k) -> size_t {
        return (size_t(i) * nt + size_t(j)) * np + size_t(((k % np) + np) % np);
      };
      S f[2][2][2], g[2][2][2], gr[2][2][2], gt[2][2][2], gp[2][2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int k = 0; k < 2; ++k) {
            int ia = a + i, jb = b + j, kc = c + k;
            f[i][j][k] = src.template ne<S>(at(ia, jb, kc));
            if (want_te) g[i][j][k] = src.template te<S>(at(ia, jb, kc));
            // vertex gradient in index units
            if (ia == 0) gr[i][j][k] = src.template ne<S>(at(1, jb, kc)) - src.template ne<S>(at(0, jb, kc));
            else if (ia == nr - 1) gr[i][j][k] = src.template ne<S>(at(nr - 1, jb, kc)) - src.template ne<S>(at(nr - 2, jb, kc));
            else gr[i][j][k] = S(0.5) * (src.template ne<S>(at(ia + 1, jb, kc)) - src.template ne<S>(at(ia - 1, jb, kc)));
            if (jb == 0) gt[i][j][k] = src.template ne<S>(at(ia, 1, kc)) - src.template ne<S>(at(ia, 0, kc));
            else if (jb == nt - 1) gt[i][j][k] = src.template ne<S>(at(ia, nt - 1, kc)) - src.template ne<S>(at(ia, nt - 2, kc));
            else gt[i][j][k] = S(0.5) * (src.template ne<S>(at(ia, jb + 1, kc)) - src.template ne<S>(at(ia, jb - 1, kc)));
            gp[i][j][k] = S(0.5) * (src.template ne<S>(at(ia, jb, kc + 1)) - src.template ne<S>(at(ia, jb, kc - 1)));
          }
      S d1, d2, d3;
      trilinear(f, u, v, w, out.ne, d1, d2, d3);
      if (want_te) trilinear(g, u, v, w, out.te, d1, d2, d3);
      S dnu, dnv, dnw;
      trilinear(gr, u, v, w, dnu, d1, d2, d3);
      trilinear(gt, u, v, w, dnv, d1, d2, d3);
      trilinear(gp, u, v, w, dnw, d1, d2, d3);
      // Beyond an edge the index is clamped: the value is held and the gradient
      // is the edge vertex's, so the force stays continuous across r_in, r_max
      // and the polar rows (a ray starts on the r_max sphere).
      (void)cr; (void)ct;
      // Chain rule to Cartesian with the spherical unit vectors.
      S st = rho / r, ctv = pos.z / r;
      V3<S> rhat = (S(1.0) / r) * pos;
      S cph(1.0), sph(0.0);
      if (!on_axis) { cph = pos.x / rho; sph = pos.y / rho; }
      V3<S> that{ctv * cph, ctv * sph, -st};
      V3<S> phat{-sph, cph, S(0.0)};
      S g_r = dnu / (r * S(dl));
      S g_t = dnv / (r * S(dth));
      out.grad = g_r * rhat + g_t * that;
      if (!on_axis) {
        S g_p = dnw / (rho * S(dph));
        out.grad = out.grad + g_p * phat;
      }
      break;
    }
    case GRID_CARTESIAN: {
      // Uniform lattice, edge-clamped; same value / gradient construction.
      const int n[3] = {m.n0, m.n1, m.n2};
      S p[3] = {pos.x, pos.y, pos.z};
      S xi[3], fr[3];
      bool cl[3];
      int base[3];
      for (int k = 0; k < 3; ++k) {
        xi[k] = clamp_index((p[k] - S(m.origin[k])) / S(m.spacing[k]), n[k], cl[k]);
        base[k] = std::min(int(std::floor(val(xi[k]))), n[k] - 2);
        fr[k] = xi[k] - S(double(base[k]));
      }
      event_mix((uint64_t(uint32_t(base[0])) << 42) ^ (uint64_t(uint32_t(base[1])) << 21) ^
                uint64_t(uint32_t(base[2])) ^ (uint64_t(cl[0]) << 61) ^ (uint64_t(cl[1]) << 62) ^
                (uint64_t(cl[2]) << 63));
      auto at = [&](int i, int j, int k) -> size_t { return (size_t(i) * n[1] + size_t(j)) * n[2] + size_t(k); };
      auto diff = [&](int ax, int i, int j, int k) -> S {
        int id[3] = {i, j, k};
        int lo[3] = {i, j, k}, hi[3] = {i, j, k};
        S scale(0.5);
        if (id[ax] == 0) { hi[ax] = 1; lo[ax] = 0; scale = S(1.0); }
        else if (id[ax] == n[ax] - 1) { hi[ax] = n[ax] - 1; lo[ax] = n[ax] - 2; scale = S(1.0); }
        else { hi[ax] = id[ax] + 1; lo[ax] = id[ax] - 1; }
        return scale * (src.template ne<S>(at(hi[0], hi[1], hi[2])) - src.template ne<S>(at(lo[0], lo[1], lo[2])));
      };
      S f[2][2][2], g[2][2][2], gx[3][2][2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int k = 0; k < 2; ++k) {
            int I = base[0] + i, J = base[1] + j, K = base[2] + k;
            f[i][j][k] = src.template ne<S>(at(I, J, K));
            if (want_te) g[i][j][k] = src.template te<S>(at(I, J, K));
            for (int ax = 0; ax < 3; ++ax) gx[ax][i][j][k] = diff(ax, I, J, K);
          }
      S d0, d1, d2;
      trilinear(f, fr[0], fr[1], fr[2], out.ne, d0, d1, d2);
      if (want_te) trilinear(g, fr[0], fr[1], fr[2], out.te, d0, d1, d2);
      S gi[3];
      for (int ax = 0; ax < 3; ++ax) trilinear(gx[ax], fr[0], fr[1], fr[2], gi[ax], d0, d1, d2);
      (void)cl;
      out.grad = {gi[0] / S(m.spacing[0]), gi[1] / S(m.spacing[1]), gi[2] / S(m.spacing[2])};
      break;
    }
    case ANALYTIC_BA: {
      S r = sqrt(dot(pos, pos));
      S ne = S(1e8) * (S(2.99) * pow(r, -16.0) + S(1.55) * pow(r, -6.0) + S(0.036) * pow(r, -1.5));
      S dne = S(1e8) * (S(-16.0 * 2.99) * pow(r, -17.0) + S(-6.0 * 1.55) * pow(r, -7.0) +
                        S(-1.5 * 0.036) * pow(r, -2.5));
      out.ne = ne;
      out.grad = (dne / r) * pos;
      out.te = S(m.t_const);
      break;
    }
    case ANALYTIC_UNIFORM:
      out.ne = S(m.a0);
      out.te = S(m.t_const);
      break;
    case ANALYTIC_SLAB:  // n_e = a0 (1 + (z - a1) / a2)
      out.ne = S(m.a0) * (S(1.0) + (pos.z - S(m.a1)) / S(m.a2));
      out.grad = {S(0.0), S(0.0), S(m.a0 / m.a2)};
      out.te = S(m.t_const);
      break;
    case ANALYTIC_LENS:  // n_e = a1 + a0 (x^2 + y^2): a quadratic lens about the z axis on a uniform background
      out.ne = S(m.a1) + S(m.a0) * (pos.x * pos.x + pos.y * pos.y);
      out.grad = {S(2.0 * m.a0) * pos.x, S(2.0 * m.a0) * pos.y, S(0.0)};
      out.te = S(m.t_const);
      break;
    default:
      break;
  }
  return out;
}

// Refractive index n = sqrt(max(1 - X, 0)), X = Xf n_e.
template <class S> S index_from_ne(const S& ne, double xf) {
  using std::sqrt;
  S n2 = S(1.0) - S(xf) * ne;
  if (val(n2) <= 0.0) return S(0.0);
  return sqrt(n2);
}

// Free-free absorption coefficient times the refractive index [cm^-1]
// (Rayleigh-Jeans thermal bremsstrahlung, Z = 1, n_i = n_e, Dulk 1985):
//   kappa * n = 9.78e-3 n_e^2 lnL / (f^2 T^{3/2}),
//   lnL = 24.5 + ln T - ln f (T >= 2e5 K), 18.2 + 1.5 ln T - ln f otherwise.
template <class S> S kappa_n(const S& ne, const S& te, double f) {
  using std::log; using std::sqrt;
  S lnl = (val(te) >= 2.0e5) ? S(24.5) + log(te) - S(std::log(f))
                             : S(18.2) + S(1.5) * log(te) - S(std::log(f));
  return S(kFFCoef) * ne * ne * lnl / (S(f * f) * te * sqrt(te));
}

// Classical fourth-order Runge-Kutta step of y' = (p, -1/2 Xf grad n_e(r)).
template <class S, class Src>
void rk4_step(const Medium& m, const Src& src, double xf, bool refr, const S& h, V3<S>& r, V3<S>& p) {
  auto force = [&](const V3<S>& x) -> V3<S> {
    if (!refr) return {S(0.0), S(0.0), S(0.0)};
    Sample<S> s = eval_medium(m, src, x, false);
    return S(-0.5 * xf) * s.grad;
  };
  V3<S> k1r = p, k1p = force(r);
  V3<S> k2r = p + (S(0.5) * h) * k1p, k2p = force(r + (S(0.5) * h) * k1r);
  V3<S> k3r = p + (S(0.5) * h) * k2p, k3p = force(r + (S(0.5) * h) * k2r);
  V3<S> k4r = p + h * k3p, k4p = force(r + h * k3r);
  r = r + (h / S(6.0)) * (k1r + S(2.0) * k2r + S(2.0) * k3r + k4r);
  p = p + (h / S(6.0)) * (k1p + S(2.0) * k2p + S(2.0) * k3p + k4p);
}

// Chord-sphere crossing: the root in [0,1] of |r + lam dr|^2 = R^2.
// outward = true picks the exit (larger) root, false the entry (smaller) root.
template <class S> S crossing(const V3<S>& r, const V3<S>& dr, double R, bool outward) {
  using std::sqrt;
  S A = dot(dr, dr), B = dot(r, dr), C = dot(r, r) - S(R * R);
  S D = B * B - A * C;
  if (val(D) < 0.0) return S(1.0);
  S lam = outward ? (-B + sqrt(D)) / A : (-B - sqrt(D)) / A;
  if (val(lam) < 0.0) return S(0.0);
  if (val(lam) > 1.0) return S(1.0);
  return lam;
}

template <class S> struct Segment { S dtau, gamma, te; };

template <class S> struct RayOut {
  S tb, tau, ln_s;
  double r_min, lam_last, bouguer_drift, ham_drift, ln_s_min;
  V3<double> exit_pos;
  int n_steps, code, flags;
};

template <class S> double vnorm(const V3<S>& a) {
  return std::sqrt(val(a.x) * val(a.x) + val(a.y) * val(a.y) + val(a.z) * val(a.z));
}

// Exact segment update of the transfer equation in brightness temperature,
// integrated toward the observer over one segment with constant kappa, T and
// d ln S/ds:  T_out = a T_in + b,  a = e^{-(dtau+gamma)},
// b = T dtau (1 - e^{-(dtau+gamma)}) / (dtau + gamma).
template <class S> S segment_apply(const Segment<S>& sg, const S& t_in) {
  using std::exp; using std::expm1;
  S x = sg.dtau + sg.gamma;
  S a = exp(-x);
  S phi = (val(x) == 0.0) ? S(1.0) : -expm1(-x) / x;
  return a * t_in + sg.te * sg.dtau * phi;
}

// One ray with the RK4 stepper (central ray + two perturbed rays per step).
template <class S, class Src>
RayOut<S> trace_rk4(const Medium& m, const Src& src, const Params& P, double f,
                    const V3<double>& r0d, const V3<double>& dird, double* path, int path_cap, int* path_len) {
  using std::log; using std::fabs; using std::sqrt;
  const double xf = (kFpCoef * kFpCoef) / (f * f);
  const bool refr = P.use_refraction != 0;
  const bool mag = refr && P.use_magnification != 0;
  RayOut<S> out{};
  V3<S> r = lift<S>(r0d);
  V3<S> d = lift<S>(dird);
  V3<S> p;
  if (refr) {
    Sample<S> s0 = eval_medium(m, src, r, false);
    p = index_from_ne(s0.ne, xf) * d;
  } else {
    p = d;
  }
  const double L0 = vnorm(cross(r, p));
  double bdrift = 0.0, hdrift = 0.0, lns_min = 0.0;
  // Carried tube: two neighbour rays launched eps = eta ds_max away from the
  // central ray across its initial direction (the Eq. 6 basis of d), each with
  // the wavevector n(start) d, stepped with the central ray's dt for the whole
  // ray; the tube cross-section at a step point is S = |(dr_a x dr_b) . p_hat|
  // with dr the separations from the central ray at equal t, and ln M of a step
  // is ln(S_{i+1} / S_i), so that the sum over the ray is ln(S_end / S_0).
  const bool carried = mag && P.carried_tube != 0;
  V3<S> ra, pa, rb, pb;
  S ln_s_prev(0.0);
  auto tube_ln_s = [&](const V3<S>& rc, const V3<S>& pc, const V3<S>& xa, const V3<S>& xb) {
    V3<S> ph = (S(1.0) / norm(pc)) * pc;
    return log(fabs(dot(cross(xa - rc, xb - rc), ph)));
  };
  if (carried) {
    V3<S> a = (std::fabs(val(d.z)) > 0.9) ? V3<S>{S(0.0), S(1.0), S(0.0)} : V3<S>{S(0.0), S(0.0), S(1.0)};
    V3<S> c1 = cross(a, d);
    V3<S> e1 = (S(1.0) / norm(c1)) * c1;
    V3<S> e2 = cross(d, e1);
    const S eps(P.eta * P.ds_max);
    ra = r + eps * e1;
    rb = r + eps * e2;
    pa = index_from_ne(eval_medium(m, src, ra, false).ne, xf) * d;
    pb = index_from_ne(eval_medium(m, src, rb, false).ne, xf) * d;
    ln_s_prev = tube_ln_s(r, p, ra, rb);
  }
  std::vector<Segment<S>> segs;
  int code = RUNNING, n_steps = 0;
  double rmin = vnorm(r), lam_last = 1.0;
  V3<double> exitp{val(r.x), val(r.y), val(r.z)};
  S tau(0.0), lns(0.0), s_arc(0.0);
  // smallest angular distance of a step point from the polar axis
  auto axis_angle = [](const V3<S>& x) {
    double rho = std::sqrt(val(x.x) * val(x.x) + val(x.y) * val(x.y));
    return std::atan2(rho, std::fabs(val(x.z)));
  };
  double min_axis = axis_angle(r);
  const bool inner = m.r_in > 0.0;
  for (int i = 0; i < P.max_steps; ++i) {
    // Step size: dt = ds_max / max(n(r_i), n_floor); arc length n dt <= ds_max.
    S dt;
    if (refr) {
      Sample<S> si = eval_medium(m, src, r, false);
      S ni = index_from_ne(si.ne, xf);
      dt = (val(ni) > P.n_floor) ? S(P.ds_max) / ni : S(P.ds_max / P.n_floor);
      event_mix(val(ni) > P.n_floor ? 1u : 2u);
    } else {
      dt = S(P.ds_max);
    }
    V3<S> r1 = r, p1 = p;
    rk4_step(m, src, xf, refr, dt, r1, p1);
    if (!(finite_s(r1.x) && finite_s(r1.y) && finite_s(r1.z) && finite_s(p1.x) && finite_s(p1.y) && finite_s(p1.z))) {
      code = NONFINITE;
      n_steps = i + 1;
      break;
    }
    // Eq. 5: propagation direction from the step chord.
    V3<S> dr = r1 - r;
    S ds = norm(dr);
    V3<S> that = (S(1.0) / ds) * dr;
    S lnM(0.0);
    if (carried) {
      rk4_step(m, src, xf, refr, dt, ra, pa);
      rk4_step(m, src, xf, refr, dt, rb, pb);
      const S ln_s = tube_ln_s(r1, p1, ra, rb);
      lnM = ln_s - ln_s_prev;
      ln_s_prev = ln_s;
    } else if (mag) {
      // Reference axis least aligned with t: z unless |t_z| is close to 1.
      V3<S> a = (std::fabs(val(that.z)) > 0.9) ? V3<S>{S(0.0), S(1.0), S(0.0)} : V3<S>{S(0.0), S(0.0), S(1.0)};
      event_mix(std::fabs(val(that.z)) > 0.9 ? 3u : 4u);
      V3<S> c1 = cross(a, that);                          // Eq. 6
      V3<S> e1 = (S(1.0) / norm(c1)) * c1;
      V3<S> e2 = cross(that, e1);
      S eps = S(P.eta) * ds;                              // Eq. 8
      V3<S> ra = r + eps * e1, pa = p;                    // Eq. 7, shared wavevector
      V3<S> rb = r + eps * e2, pb = p;
      rk4_step(m, src, xf, refr, dt, ra, pa);
      rk4_step(m, src, xf, refr, dt, rb, pb);
      V3<S> d1 = ra - r1, d2 = rb - r1;                   // Eq. 9
      S area = fabs(dot(cross(d1, d2), that));            // Eq. 10 without the 1/2
      event_mix(val(dot(cross(d1, d2), that)) < 0.0 ? 5u : 6u);
      S M = area / (eps * eps);                           // Eq. 11
      lnM = log(M);
    }
    // Termination on the two spheres; the last chord is truncated at the crossing.
    S lam(1.0);
    double r1n2 = val(dot(r1, r1));
    if (inner && r1n2 <= m.r_in * m.r_in) {
      code = HIT_INNER;
      lam = crossing(r, dr, m.r_in, false);
    } else if (r1n2 >= m.r_max * m.r_max && i >= 1) {
      code = EXIT_OUTER;
      lam = crossing(r, dr, m.r_max, true);
    } else if (i + 1 == P.max_steps) {
      code = MAX_STEPS;
    }
    // Segment coefficients at the chord midpoint.
    V3<S> rm = r + (S(0.5) * lam) * dr;
    Sample<S> sm = eval_medium(m, src, rm, true);
    S dtau = P.no_absorption ? S(0.0) : kappa_n(sm.ne, sm.te, f) * S(kRsunCm) * lam * dt;
    S gamma = -(lam * lnM);
    segs.push_back({dtau, gamma, sm.te});
    tau = tau + dtau;
    lns = lns + lam * lnM;
    lns_min = std::min(lns_min, val(lns));
    s_arc = s_arc + lam * ds;
    if (path && path_len && *path_len < path_cap) {
      V3<S> pe = r + lam * dr;
      double* rec = path + size_t(*path_len) * kPathStride;
      rec[0] = val(pe.x); rec[1] = val(pe.y); rec[2] = val(pe.z);
      rec[3] = val(s_arc); rec[4] = val(lnM); rec[5] = val(lnM) / val(ds);
      rec[6] = val(tau); rec[7] = val(sm.ne); rec[8] = val(sm.te);
      rec[9] = val(dtau); rec[10] = val(gamma); rec[11] = val(dt);
      ++*path_len;
    }
    if (code != RUNNING) {
      V3<S> pe = r + lam * dr;
      exitp = {val(pe.x), val(pe.y), val(pe.z)};
      rmin = std::min(rmin, vnorm(pe));
      lam_last = val(lam);
      n_steps = i + 1;
      break;
    }
    r = r1;
    p = p1;
    rmin = std::min(rmin, vnorm(r));
    min_axis = std::min(min_axis, axis_angle(r));
    if (L0 > 0.0) bdrift = std::max(bdrift, std::fabs(vnorm(cross(r, p)) - L0) / L0);
    if (refr && std::is_same<S, double>::value) {  // diagnostic only: kept off the AD tapes
      Sample<S> sh = eval_medium(m, src, r, false);
      hdrift = std::max(hdrift, std::fabs(val(dot(p, p)) + xf * val(sh.ne) - 1.0));
    }
  }
  if (code == NONFINITE) exitp = {val(r.x), val(r.y), val(r.z)};
  // Transfer from the far end back toward the observer (Sec. 3.2, Fig. 5).
  S T = (code == HIT_INNER) ? S(P.tb_inner) : S(P.tb_sky);
  for (int i = int(segs.size()) - 1; i >= 0; --i) T = segment_apply(segs[size_t(i)], T);
  out.tb = T;
  out.tau = tau;
  out.ln_s = lns;
  out.r_min = rmin;
  out.lam_last = lam_last;
  out.exit_pos = exitp;
  out.n_steps = n_steps;
  out.code = code;
  out.flags = 0;
  out.bouguer_drift = bdrift;
  out.ham_drift = hdrift;
  out.ln_s_min = lns_min;
  if ((code == EXIT_OUTER || code == HIT_INNER) && (lam_last < 1e-4 || lam_last > 1.0 - 1e-4))
    out.flags |= MARGINAL;
  // Near the polar axis of a spherical grid the theta rows are clamped and the
  // azimuthal derivative is divided by rho -> 0: the force is singular there and
  // a ray passing through it is ill-conditioned.
  if (m.kind == GRID_SPHERICAL_LOGR && min_axis < 2.0 * (0.5 * kPi / double(m.n1))) out.flags |= POLAR;
  return out;
}

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) with error control (central ray; physics reference).
// ---------------------------------------------------------------------------
struct State6 { V3<double> r, p; };

static State6 dp_deriv(const Medium& m, double xf, bool refr, const State6& y) {
  PlainSource src{&m};
  State6 d;
  d.r = y.p;
  if (refr) {
    Sample<double> s = eval_medium(m, src, y.r, false);
    d.p = (-0.5 * xf) * s.grad;
  } else {
    d.p = {0, 0, 0};
  }
  return d;
}
static State6 axpy(const State6& y, double h, std::initializer_list<std::pair<double, const State6*>> terms) {
  State6 o = y;
  for (auto& t : terms) {
    o.r = o.r + (h * t.first) * t.second->r;
    o.p = o.p + (h * t.first) * t.second->p;
  }
  return o;
}
// One Dormand-Prince step; returns the 5th-order solution and the error estimate.
static void dp_step(const Medium& m, double xf, bool refr, const State6& y, double h, State6& y5, double err[6]) {
  State6 k1 = dp_deriv(m, xf, refr, y);
  State6 k2 = dp_deriv(m, xf, refr, axpy(y, h, {{1.0 / 5, &k1}}));
  State6 k3 = dp_deriv(m, xf, refr, axpy(y, h, {{3.0 / 40, &k1}, {9.0 / 40, &k2}}));
  State6 k4 = dp_deriv(m, xf, refr, axpy(y, h, {{44.0 / 45, &k1}, {-56.0 / 15, &k2}, {32.0 / 9, &k3}}));
  State6 k5 = dp_deriv(m, xf, refr, axpy(y, h, {{19372.0 / 6561, &k1}, {-25360.0 / 2187, &k2},
                                               {64448.0 / 6561, &k3}, {-212.0 / 729, &k4}}));
  State6 k6 = dp_deriv(m, xf, refr, axpy(y, h, {{9017.0 / 3168, &k1}, {-355.0 / 33, &k2}, {46732.0 / 5247, &k3},
                                               {49.0 / 176, &k4}, {-5103.0 / 18656, &k5}}));
  y5 = axpy(y, h, {{35.0 / 384, &k1}, {500.0 / 1113, &k3}, {125.0 / 192, &k4}, {-2187.0 / 6784, &k5},
                   {11.0 / 84, &k6}});
  State6 k7 = dp_deriv(m, xf, refr, y5);
  State6 y4 = axpy(y, h, {{5179.0 / 57600, &k1}, {7571.0 / 16695, &k3}, {393.0 / 640, &k4},
                          {-92097.0 / 339200, &k5}, {187.0 / 2100, &k6}, {1.0 / 40, &k7}});
  double e[6] = {y5.r.x - y4.r.x, y5.r.y - y4.r.y, y5.r.z - y4.r.z, y5.p.x - y4.p.x, y5.p.y - y4.p.y, y5.p.z - y4.p.z};
  for (int i = 0; i < 6; ++i) err[i] = e[i];
}

static RayOut<double> trace_dp54(const Medium& m, const Params& P, double f, const V3<double>& r0,
                                 const V3<double>& dir, double* path, int path_cap, int* path_len) {
  PlainSource src{&m};
  const double xf = (kFpCoef * kFpCoef) / (f * f);
  const bool refr = P.use_refraction != 0;
  RayOut<double> out{};
  State6 y;
  y.r = r0;
  if (refr) {
    Sample<double> s0 = eval_medium(m, src, r0, false);
    y.p = index_from_ne(s0.ne, xf) * dir;
  } else {
    y.p = dir;
  }
  const double L0 = vnorm(cross(y.r, y.p));
  double bdrift = 0, hdrift = 0;
  std::vector<Segment<double>> segs;
  int code = RUNNING, n_steps = 0;
  double rmin = vnorm(y.r), lam_last = 1.0, tau = 0, s_arc = 0;
  V3<double> exitp = y.r;
  const bool inner = m.r_in > 0.0;
  double h = P.ds_max;
  for (int i = 0; i < P.max_steps; ++i) {
    double hmax;
    if (refr) {
      double ni = index_from_ne(eval_medium(m, src, y.r, false).ne, xf);
      hmax = P.ds_max / std::max(ni, P.n_floor);
    } else {
      hmax = P.ds_max;
    }
    h = std::min(h, hmax);
    State6 y5;
    double e[6];
    for (int tries = 0;; ++tries) {
      dp_step(m, xf, refr, y, h, y5, e);
      double en = 0;
      double yy[6] = {y.r.x, y.r.y, y.r.z, y.p.x, y.p.y, y.p.z};
      double zz[6] = {y5.r.x, y5.r.y, y5.r.z, y5.p.x, y5.p.y, y5.p.z};
      for (int k = 0; k < 6; ++k)
        en = std::max(en, std::fabs(e[k]) / (P.dp_atol + P.dp_rtol * std::max(std::fabs(yy[k]), std::fabs(zz[k]))));
      double fac = (en > 0) ? 0.9 * std::pow(en, -0.2) : 5.0;
      fac = std::min(5.0, std::max(0.2, fac));
      if (en <= 1.0 || tries > 60) {
        // turning point inside the accepted step: refine r_min by bisection on
        // r.p using single Dormand-Prince steps of a fraction of h from y.
        if (refr && dot(y.r, y.p) < 0.0 && dot(y5.r, y5.p) >= 0.0) {
          double lo = 0.0, hi = 1.0;
          for (int it = 0; it < 60; ++it) {
            double mid = 0.5 * (lo + hi);
            State6 ym; double em[6];
            dp_step(m, xf, refr, y, mid * h, ym, em);
            if (dot(ym.r, ym.p) < 0.0) lo = mid; else hi = mid;
          }
          State6 ym; double em[6];
          dp_step(m, xf, refr, y, 0.5 * (lo + hi) * h, ym, em);
          rmin = std::min(rmin, vnorm(ym.r));
        }
        double hused = h;
        h = std::min(h * fac, 1e9);
        V3<double> dr = y5.r - y.r;
        double lam = 1.0;
        double r1n2 = dot(y5.r, y5.r);
        if (inner && r1n2 <= m.r_in * m.r_in) { code = HIT_INNER; lam = crossing(y.r, dr, m.r_in, false); }
        else if (r1n2 >= m.r_max * m.r_max && i >= 1) { code = EXIT_OUTER; lam = crossing(y.r, dr, m.r_max, true); }
        else if (i + 1 == P.max_steps) code = MAX_STEPS;
        V3<double> rm = y.r + (0.5 * lam) * dr;
        Sample<double> sm = eval_medium(m, src, rm, true);
        double dtau = P.no_absorption ? 0.0 : kappa_n(sm.ne, sm.te, f) * kRsunCm * lam * hused;
        segs.push_back({dtau, 0.0, sm.te});
        tau += dtau;
        s_arc += lam * norm(dr);
        if (path && path_len && *path_len < path_cap) {
          V3<double> pe = y.r + lam * dr;
          double* rec = path + size_t(*path_len) * kPathStride;
          rec[0] = pe.x; rec[1] = pe.y; rec[2] = pe.z; rec[3] = s_arc; rec[4] = 0; rec[5] = 0;
          rec[6] = tau; rec[7] = sm.ne; rec[8] = sm.te; rec[9] = dtau; rec[10] = 0; rec[11] = hused;
          ++*path_len;
        }
        if (code != RUNNING) {
          V3<double> pe = y.r + lam * dr;
          exitp = pe;
          rmin = std::min(rmin, vnorm(pe));
          lam_last = lam;
          n_steps = i + 1;
        } else {
          y = y5;
          rmin = std::min(rmin, vnorm(y.r));
          if (L0 > 0) bdrift = std::max(bdrift, std::fabs(vnorm(cross(y.r, y.p)) - L0) / L0);
          if (refr) hdrift = std::max(hdrift, std::fabs(dot(y.p, y.p) + xf * eval_medium(m, src, y.r, false).ne - 1.0));
        }
        break;
      }
      h *= fac;
    }
    if (code != RUNNING) break;
  }
  double T = (code == HIT_INNER) ? P.tb_inner : P.tb_sky;
  for (int i = int(segs.size()) - 1; i >= 0; --i) T = segment_apply(segs[size_t(i)], T);
  out.tb = T; out.tau = tau; out.ln_s = 0; out.r_min = rmin; out.lam_last = lam_last;
  out.exit_pos = exitp; out.n_steps = n_steps; out.code = code; out.flags = 0;
  out.bouguer_drift = bdrift; out.ham_drift = hdrift; out.ln_s_min = 0.0;
  return out;
}

// ---------------------------------------------------------------------------
// Launch geometry (Sec. 3.2): parallel rays from the observer's image plane.
// Sun->observer unit vector o, image axes u = up x o (normalised), v = o x u;
// pixel centres -h + (j + 1/2) 2h/n; start on the r_max sphere, direction -o.
// ---------------------------------------------------------------------------
struct Launch { V3<double> r0, dir; double b; };

static void image_axes(const Image& im, V3<double>& o, V3<double>& u, V3<double>& v) {
  o = {im.obs_dir[0], im.obs_dir[1], im.obs_dir[2]};
  o = (1.0 / norm(o)) * o;
  V3<double> up{im.up[0], im.up[1], im.up[2]};
  u = cross(up, o);
  u = (1.0 / norm(u)) * u;
  v = cross(o, u);
}

static Launch pixel_launch(const Image& im, double r_max, int ju, int iv, double du_extra) {
  V3<double> o, u, v;
  image_axes(im, o, u, v);
  double pu = -im.half_u + (ju + 0.5) * 2.0 * im.half_u / im.nu + du_extra;
  double pv = -im.half_v + (iv + 0.5) * 2.0 * im.half_v / im.nv;
  double b2 = pu * pu + pv * pv;
  Launch L;
  L.b = std::sqrt(b2);
  double x0 = (b2 < r_max * r_max) ? std::sqrt(r_max * r_max - b2) : 0.0;
  L.r0 = x0 * o + pu * u + pv * v;
  L.dir = (-1.0) * o;
  return L;
}

static void fill_result(const RayOut<double>& ro, Result& r) {
  r.tb = ro.tb; r.tau = ro.tau; r.ln_s_end = ro.ln_s; r.r_min = ro.r_min;
  r.exit_pos[0] = ro.exit_pos.x; r.exit_pos[1] = ro.exit_pos.y; r.exit_pos[2] = ro.exit_pos.z;
  r.lam_last = ro.lam_last; r.n_steps = ro.n_steps; r.code = ro.code; r.flags = ro.flags;
  r.bouguer_drift = ro.bouguer_drift; r.ham_drift = ro.ham_drift; r.ln_s_min = ro.ln_s_min; r._pad = 0;
  r.twin_dexit = -1.0;
  r.event_hash = 0;
}

static RayOut<double> trace_any(const Medium& m, const Params& P, double f, const V3<double>& r0,
                                const V3<double>& dir, double* path, int cap, int* plen) {
  if (P.stepper == 1) return trace_dp54(m, P, f, r0, dir, path, cap, plen);
  PlainSource src{&m};
  return trace_rk4<double>(m, src, P, f, r0, dir, path, cap, plen);
}

// Grazing / ill-conditioned classification of a traced image ray.
static int grazing_flags(const Medium& m, const Params& P, const Image& im, double f, int ju, int iv,
                         const RayOut<double>& ro, double* twin_dexit) {
  int fl = 0;
  *twin_dexit = -1.0;
  if (ro.code == HIT_INNER) {
    // incidence at the inner sphere: angle between the exit point's radial
    // direction and the final chord, from a re-trace that records the path
    std::vector<double> path(size_t(ro.n_steps + 2) * kPathStride);
    int plen = 0;
    Launch L = pixel_launch(im, m.r_max, ju, iv, 0.0);
    trace_any(m, P, f, L.r0, L.dir, path.data(), ro.n_steps + 2, &plen);
    if (plen >= 2) {
      const double* a = &path[size_t(plen - 2) * kPathStride];
      const double* b = &path[size_t(plen - 1) * kPathStride];
      V3<double> t{b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      V3<double> e{b[0], b[1], b[2]};
      double c = std::fabs(dot(t, e)) / (norm(t) * norm(e));
      if (c < 0.1) fl |= GRAZING;
    }
  } else if (ro.code != MISS && m.r_in > 0.0 && ro.r_min < m.r_in + 0.01) {
    fl |= GRAZING;
  }
  if (P.twin_check && ro.code != MISS) {
    Launch T = pixel_launch(im, m.r_max, ju, iv, 1e-6);
    RayOut<double> tw = trace_any(m, P, f, T.r0, T.dir, nullptr, 0, nullptr);
    double dx = tw.exit_pos.x - ro.exit_pos.x, dy = tw.exit_pos.y - ro.exit_pos.y, dz = tw.exit_pos.z - ro.exit_pos.z;
    const double move = std::sqrt(dx * dx + dy * dy + dz * dz);
    *twin_dexit = (tw.code != ro.code) ? std::numeric_limits<double>::infinity() : move;
    if (tw.code != ro.code || move > P.twin_exit_tol) fl |= GRAZING;
  }
  return fl;
}

template <class F> static void parallel_for(int n, int n_threads, F&& fn) {
  if (n_threads <= 1 || n < 2) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next(0);
  const int chunk = 4;
  std::vector<std::thread> pool;
  for (int t = 0; t < n_threads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int s = next.fetch_add(chunk);
        if (s >= n) break;
        for (int i = s; i < std::min(n, s + chunk); ++i) fn(i);
      }
    });
  for (auto& th : pool) th.join();
}

}  // namespace orc

using namespace orc;

extern "C" {

int orc_abi_version(void) { return 1; }

// Trace explicitly launched rays: r0 and dir are [n][3] (dir need not be unit).
int orc_trace_launch(const Medium* m, const Params* P, double freq, int n, const double* r0, const double* dir,
                     Result* out, double* path, int path_cap, int* path_len, int n_threads) {
  if (!m || !P || !r0 || !dir || !out || n < 0) return 1;
  if (path && n != 1) return 1;
  parallel_for(n, path ? 1 : n_threads, [&](int i) {
    V3<double> a{r0[3 * i], r0[3 * i + 1], r0[3 * i + 2]};
    V3<double> d{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
    d = (1.0 / norm(d)) * d;
    if (path_len) *path_len = 0;
    RayOut<double> ro = trace_any(*m, *P, freq, a, d, path, path_cap, path_len);
    fill_result(ro, out[i]);
  });
  return 0;
}

// Trace image pixels (flat index = iv * nu + ju) at one frequency.
int orc_trace_pixels(const Medium* m, const Params* P, const Image* im, double freq, int n, const int32_t* pix,
                     Result* out, int n_threads) {
  if (!m || !P || !im || !pix || !out || n < 0) return 1;
  parallel_for(n, n_threads, [&](int i) {
    int ju = pix[i] % im->nu, iv = pix[i] / im->nu;
    Launch L = pixel_launch(*im, m->r_max, ju, iv, 0.0);
    Result& r = out[i];
    if (L.b >= m->r_max) {
      std::memset(&r, 0, sizeof(Result));
      r.tb = P->tb_sky; r.code = MISS; r.n_steps = 0;
      r.exit_pos[0] = L.r0.x; r.exit_pos[1] = L.r0.y; r.exit_pos[2] = L.r0.z;
      r.r_min = L.b; r.lam_last = 1.0;
      return;
    }
    uint64_t hash = 0xcbf29ce484222325ull;
    event_hash_ref() = &hash;
    RayOut<double> ro = trace_any(*m, *P, freq, L.r0, L.dir, nullptr, 0, nullptr);
    event_hash_ref() = nullptr;
    fill_result(ro, r);
    hash ^= (uint64_t(uint32_t(ro.n_steps)) << 8) ^ uint64_t(uint32_t(ro.code));
    r.event_hash = hash;
    r.flags |= grazing_flags(*m, *P, *im, freq, ju, iv, ro, &r.twin_dexit);
  });
  return 0;
}

// One image pixel with its recorded path (kPathStride doubles per step).
int orc_trace_pixel_path(const Medium* m, const Params* P, const Image* im, double freq, int pix, Result* out,
                         double* path, int path_cap, int* path_len) {
  int ju = pix % im->nu, iv = pix / im->nu;
  Launch L = pixel_launch(*im, m->r_max, ju, iv, 0.0);
  *path_len = 0;
  if (L.b >= m->r_max) {
    std::memset(out, 0, sizeof(Result));
    out->tb = P->tb_sky; out->code = MISS;
    return 0;
  }
  RayOut<double> ro = trace_any(*m, *P, freq, L.r0, L.dir, path, path_cap, path_len);
  fill_result(ro, *out);
  return 0;
}

// Medium probe: n_e, grad n_e, T at n points [n][3] -> out [n][5].
int orc_eval_medium(const Medium* m, int n, const double* pos, double* out) {
  PlainSource src{m};
  for (int i = 0; i < n; ++i) {
    V3<double> x{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    Sample<double> s = eval_medium(*m, src, x, true);
    out[5 * i] = s.ne; out[5 * i + 1] = s.grad.x; out[5 * i + 2] = s.grad.y; out[5 * i + 3] = s.grad.z;
    out[5 * i + 4] = s.te;
  }
  return 0;
}

// Free-free coefficient probe: kappa*n [cm^-1] for n (ne, T) pairs at frequency f.
int orc_kappa_n(int n, const double* ne, const double* te, double f, double* out) {
  for (int i = 0; i < n; ++i) out[i] = kappa_n(ne[i], te[i], f);
  return 0;
}

// Directional derivative of sum_i w_i T_b,i over image pixels, along
// (vn, vt) in (ln n_e, ln T) per vertex, by forward-mode dual numbers.
int orc_dual_loss(const Medium* m, const Params* P, const Image* im, int n_freq, const double* freqs,
                  const float* w, const double* vn, const double* vt, double* loss, double* dloss, int n_threads) {
  const int npx = im->nu * im->nv;
  const int n = npx * n_freq;
  std::vector<double> lv(size_t(n), 0.0), ld(size_t(n), 0.0);
  DualSource src{m, vn, vt};
  parallel_for(n, n_threads, [&](int k) {
    int fi = k / npx, px = k % npx;
    int ju = px % im->nu, iv = px / im->nu;
    if (w[k] == 0.0f) return;  // contributes nothing
    Launch L = pixel_launch(*im, m->r_max, ju, iv, 0.0);
    if (L.b >= m->r_max) { lv[size_t(k)] = w[k] * P->tb_sky; return; }
    RayOut<Dual> ro = trace_rk4<Dual>(*m, src, *P, freqs[fi], L.r0, L.dir, nullptr, 0, nullptr);
    lv[size_t(k)] = double(w[k]) * ro.tb.v;
    ld[size_t(k)] = double(w[k]) * ro.tb.d;
  });
  double s = 0, sd = 0;
  for (int k = 0; k < n; ++k) { s += lv[size_t(k)]; sd += ld[size_t(k)]; }
  *loss = s;
  *dloss = sd;
  return 0;
}

// Gradient of sum_k w_k T_b,k over the rays of an image stack (k = freq * npx +
// pixel; rays with w_k = 0 are skipped) w.r.t. ln n_e and ln T at every vertex,
// by reverse-mode sweeps of per-ray tapes.  gne / gte [n0 n1 n2] are overwritten.
int orc_grad_loss(const Medium* m, const Params* P, const Image* im, int n_freq, const double* freqs,
                  const float* w, double* loss, double* gne, double* gte, int n_threads) {
  if (!m || !P || !im || !freqs || !w || !loss || !gne || !gte || n_freq < 1) return 1;
  if (m->kind != GRID_SPHERICAL_LOGR && m->kind != GRID_CARTESIAN) return 1;
  const int npx = im->nu * im->nv;
  const int n = npx * n_freq;
  const size_t nv = size_t(m->n0) * m->n1 * m->n2;
  if (n_threads < 1) n_threads = 1;
  const size_t nth = size_t(n_threads);
  std::vector<std::vector<double>> part_ne(nth), part_te(nth);
  std::vector<double> part_loss(size_t(n_threads), 0.0);
  std::atomic<int> next(0);
  RevSource src{m};
  auto worker = [&](int tid) {
    Tape tape;
    tape_ref() = &tape;
    std::vector<double> adj;
    std::vector<double>& g1 = part_ne[size_t(tid)];
    std::vector<double>& g2 = part_te[size_t(tid)];
    g1.assign(nv, 0.0);
    g2.assign(nv, 0.0);
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      if (w[k] == 0.0f) continue;
      const int fi = k / npx, px = k % npx;
      Launch L = pixel_launch(*im, m->r_max, px % im->nu, px / im->nu, 0.0);
      if (L.b >= m->r_max) { part_loss[size_t(tid)] += double(w[k]) * P->tb_sky; continue; }
      tape.nodes.clear();
      RayOut<Rev> ro = trace_rk4<Rev>(*m, src, *P, freqs[fi], L.r0, L.dir, nullptr, 0, nullptr);
      part_loss[size_t(tid)] += double(w[k]) * ro.tb.v;
      if (ro.code != NONFINITE) rev_sweep(ro.tb, double(w[k]), g1.data(), g2.data(), adj);
    }
    tape_ref() = nullptr;
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < n_threads; ++t) pool.emplace_back(worker, t);
  for (auto& th : pool) th.join();
  double s = 0.0;
  for (int t = 0; t < n_threads; ++t) s += part_loss[size_t(t)];
  *loss = s;
  for (size_t v = 0; v < nv; ++v) {
    double a = 0.0, b = 0.0;
    for (int t = 0; t < n_threads; ++t) { a += part_ne[size_t(t)][v]; b += part_te[size_t(t)][v]; }
    gne[v] = a;
    gte[v] = b;
  }
  return 0;
}

}  // extern "C"
