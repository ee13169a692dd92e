// Kernels of the reverse mode: the forward pass with per-ray checkpoints, the
// reverse sweeps, and the gather that turns channel adjoints into
// d loss / d ln n_e and d loss / d ln T per vertex.
#include <hip/hip_runtime.h>

#include "rt_internal.hpp"
#include "rt_adjoint.hpp"

namespace rt {

// Tile of the batch -> (image, pixel) of a lane; false for a lane outside a
// ragged image.
__device__ __forceinline__ bool tile_pixel(const TraceArgs& a, int t, int lane, int& img, int& pix) {
  img = t / a.tiles_per_image;
  const int rem = t - img * a.tiles_per_image;
  const int ty = rem / a.tiles_u, tx = rem - ty * a.tiles_u;
  const int i = ty * kTile + (lane >> 3), j = tx * kTile + (lane & 7);
  pix = i * a.nu + j;
  return i < a.nv && j < a.nu;
}

// Forward pass of the adjoint: one wave per tile of the batch, one lane per ray,
// two waves per SIMD like the forward kernels.  Per-ray checkpoints and the
// sweep record go to the ray's column rid = 64 (tile - tile0) + lane.
template <int KIND, int MODE>
__global__ __launch_bounds__(256, 2) void k_adjoint_forward(AdjointArgs aa) {
  __shared__ float4 lds_c[4][8][kWaveLanes];
  __shared__ float lds_t[4][8][kWaveLanes];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tl = blockIdx.x * 4 + wave;
  double loss = 0.0;
  if (tl < aa.n_tiles) {
    CellCache C;
    C.key = -1;
    C.c = &lds_c[wave][0][lane];
    C.t = &lds_t[wave][0][lane];
    const int rid = tl * kWaveLanes + lane;
    int img, pix;
    if (tile_pixel(aa.t, aa.tile0 + tl, lane, img, pix)) adjoint_forward_ray<KIND, MODE>(aa, img, pix, rid, C, loss);
    else aa.meta[rid] = 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
  if (lane == 0 && tl < aa.n_tiles) unsafeAtomicAdd(aa.loss, loss);
}

// Reverse sweeps: a wave claims one tile of the batch at a time from a global
// counter; each lane sweeps its ray backward from the ray's checkpoints.
// The tracing mode (line of sight, refraction, refraction with magnification)
// is a template parameter: one kernel per mode, with no branch on the call's
// flags anywhere in the per-ray code.  The chunk record is indexed by the lane's
// global slot.
template <int KIND, int MODE>
__global__ __launch_bounds__(256, 1) void k_adjoint(AdjointArgs aa) {
  __shared__ float4 lds_c[4][8][kWaveLanes];
  __shared__ float lds_t[4][8][kWaveLanes];
  __shared__ float lds_g[4][8 * kGradChannels][kWaveLanes];
  __shared__ float lds_log[4][kLogEntries * kLogWords][kWaveLanes];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  CellCache C;
  C.key = -1;
  C.c = &lds_c[wave][0][lane];
  C.t = &lds_t[wave][0][lane];
  GradAcc A;
  A.key = -1;
  A.v = &lds_g[wave][0][lane];
  for (int k = 0; k < 8 * kGradChannels; ++k) A.v[k * kWaveLanes] = 0.0f;
  float* lg = &lds_log[wave][0][lane];
  for (;;) {
    unsigned t = 0;
    if (lane == 0) t = atomicAdd(aa.counter, 1u);
    t = (unsigned)__shfl((int)t, 0);
    if (t >= (unsigned)aa.n_tiles) break;
    int img, pix;
    if (tile_pixel(aa.t, aa.tile0 + int(t), lane, img, pix))
      adjoint_reverse_ray<KIND, MODE>(aa, img, pix, int(t) * kWaveLanes + lane, slot, C, A, lg);
  }
  grad_flush(aa.t.g, A, aa.gacc);
}

// d channel(a') / d n_e(a) for the index-space central difference along a
// clamped axis of n vertices (one-sided at the two edges).
__device__ __forceinline__ double diff_coef(int ap, int a, int n) {
  if (ap == 0) return (a == 1 ? 1.0 : 0.0) - (a == 0 ? 1.0 : 0.0);
  if (ap == n - 1) return (a == n - 1 ? 1.0 : 0.0) - (a == n - 2 ? 1.0 : 0.0);
  return (a == ap + 1 ? 0.5 : 0.0) - (a == ap - 1 ? 0.5 : 0.0);
}

// Per vertex (C-order [n0][n1][n2]): gather the adjoints of every packed
// channel that depends on its n_e (its value, the central differences of its
// neighbours, the periodic wrap column) and scale by the value for the ln.
__global__ void k_unpack_grad(DevGeom g, const float4* __restrict__ nfg, const float* __restrict__ te,
                              const double* __restrict__ gacc, float* __restrict__ gne, float* __restrict__ gte) {
  const long long total = (long long)g.n0 * g.n1 * g.n2;
  const bool periodic = g.kind == RT_GRID_SPHERICAL_LOGR;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < total;
       v += (long long)gridDim.x * blockDim.x) {
    const int c = int(v % g.n2);
    const long long ab = v / g.n2;
    const int b = int(ab % g.n1);
    const int a = int(ab / g.n1);
    auto packed = [&](int i, int j, int k) -> long long { return ((long long)i * g.n1 + j) * g.n2p + k; };
    auto ch = [&](int i, int j, int k, int q) -> double {
      double s = gacc[packed(i, j, k) * kGradChannels + q];
      if (periodic && k == 0) s += gacc[packed(i, j, g.n2) * kGradChannels + q];
      return s;
    };
    double nb = ch(a, b, c, 0);
    for (int ap = a - 1; ap <= a + 1; ++ap)
      if (ap >= 0 && ap < g.n0) nb += diff_coef(ap, a, g.n0) * ch(ap, b, c, 1);
    for (int bp = b - 1; bp <= b + 1; ++bp)
      if (bp >= 0 && bp < g.n1) nb += diff_coef(bp, b, g.n1) * ch(a, bp, c, 2);
    if (periodic) {
      const int cm = (c == 0) ? g.n2 - 1 : c - 1;
      const int cp = (c == g.n2 - 1) ? 0 : c + 1;
      nb += 0.5 * ch(a, b, cm, 3) - 0.5 * ch(a, b, cp, 3);
    } else {
      for (int cq = c - 1; cq <= c + 1; ++cq)
        if (cq >= 0 && cq < g.n2) nb += diff_coef(cq, c, g.n2) * ch(a, b, cq, 3);
    }
    const long long p = packed(a, b, c);
    gne[v] = float(double(nfg[p].x) * nb);
    gte[v] = float(double(te[p]) * ch(a, b, c, 4));
  }
}

static int grid_for(long long n, int threads) {
  long long b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return int(b);
}

template <int KIND>
static hipError_t launch_adjoint_forward_kind(const AdjointArgs& a, hipStream_t s) {
  const bool refr = (a.t.flags & RT_USE_REFRACTION) != 0;
  const bool mag = refr && (a.t.flags & RT_USE_MAGNIFICATION) != 0;
  const int blocks = (a.n_tiles + 3) / 4;
  if (mag) hipLaunchKernelGGL((k_adjoint_forward<KIND, kModeFull>), dim3(blocks), dim3(256), 0, s, a);
  else if (refr) hipLaunchKernelGGL((k_adjoint_forward<KIND, kModeNoMag>), dim3(blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_adjoint_forward<KIND, kModeLos>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adjoint_forward(const AdjointArgs& a, hipStream_t s) {
  if (a.t.g.kind == RT_GRID_SPHERICAL_LOGR) return launch_adjoint_forward_kind<RT_GRID_SPHERICAL_LOGR>(a, s);
  return launch_adjoint_forward_kind<RT_GRID_CARTESIAN>(a, s);
}

template <int KIND>
static hipError_t launch_adjoint_kind(const AdjointArgs& a, int blocks, hipStream_t s) {
  const bool refr = (a.t.flags & RT_USE_REFRACTION) != 0;
  const bool mag = refr && (a.t.flags & RT_USE_MAGNIFICATION) != 0;
  if (mag) hipLaunchKernelGGL((k_adjoint<KIND, kModeFull>), dim3(blocks), dim3(256), 0, s, a);
  else if (refr) hipLaunchKernelGGL((k_adjoint<KIND, kModeNoMag>), dim3(blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_adjoint<KIND, kModeLos>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjointArgs& a, int blocks, hipStream_t s) {
  if (a.t.g.kind == RT_GRID_SPHERICAL_LOGR) return launch_adjoint_kind<RT_GRID_SPHERICAL_LOGR>(a, blocks, s);
  return launch_adjoint_kind<RT_GRID_CARTESIAN>(a, blocks, s);
}

hipError_t launch_unpack_grad(const DevGeom& g, const float4* nfg, const float* te, const double* gacc,
                              float* grad_ln_ne, float* grad_ln_te, hipStream_t s) {
  const long long total = (long long)g.n0 * g.n1 * g.n2;
  hipLaunchKernelGGL(k_unpack_grad, dim3(grid_for(total, 256)), dim3(256), 0, s, g, nfg, te, gacc, grad_ln_ne,
                     grad_ln_te);
  return hipGetLastError();
}

int adjoint_blocks_per_cu(int kind) {
  int n = 0;
  const hipError_t e =
      (kind == RT_GRID_SPHERICAL_LOGR)
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adjoint<RT_GRID_SPHERICAL_LOGR, kModeFull>, 256, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adjoint<RT_GRID_CARTESIAN, kModeFull>, 256, 0);
  if (e != hipSuccess || n < 1) n = 1;
  return n;
}

}  // namespace rt
