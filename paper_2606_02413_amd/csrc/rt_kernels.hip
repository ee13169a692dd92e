// Kernels: model staging, value validation, and the ray tracer in its two
// launch forms (one launch per image, or one persistent launch with lane refill).
#include <hip/hip_runtime.h>

#include "rt_internal.hpp"
#include "rt_trace.hpp"

namespace rt {

// ---------------------------------------------------------------------------
// Model staging: C-order [n0][n1][n2] n_e, T  ->  packed rows of n2p vertices
// holding (n_e, dn/dxi_0, dn/dxi_1, dn/dxi_2) and T.  The index-space vertex
// gradient is the central difference (one-sided at non-periodic edges); for
// spherical grids the phi axis is periodic and row element n2 repeats element 0,
// so a cell's two phi corners are always adjacent in memory.
// ---------------------------------------------------------------------------
__global__ void k_pack(DevGeom g, const float* __restrict__ ne, const float* __restrict__ te, float4* __restrict__ nfg,
                       float* __restrict__ te_out) {
  const long long total = (long long)g.n0 * g.n1 * g.n2p;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int cp = int(idx % g.n2p);
    const long long ab = idx / g.n2p;
    const int b = int(ab % g.n1);
    const int a = int(ab / g.n1);
    const bool periodic = g.kind == RT_GRID_SPHERICAL_LOGR;
    const int c = (cp == g.n2) ? 0 : cp;  // only reached for the periodic wrap column
    auto at = [&](int i, int j, int k) -> float { return ne[((long long)i * g.n1 + j) * g.n2 + k]; };
    float d0, d1, d2;
    if (a == 0) d0 = at(1, b, c) - at(0, b, c);
    else if (a == g.n0 - 1) d0 = at(g.n0 - 1, b, c) - at(g.n0 - 2, b, c);
    else d0 = 0.5f * (at(a + 1, b, c) - at(a - 1, b, c));
    if (b == 0) d1 = at(a, 1, c) - at(a, 0, c);
    else if (b == g.n1 - 1) d1 = at(a, g.n1 - 1, c) - at(a, g.n1 - 2, c);
    else d1 = 0.5f * (at(a, b + 1, c) - at(a, b - 1, c));
    if (periodic) {
      const int cm = (c == 0) ? g.n2 - 1 : c - 1;
      const int cq = (c == g.n2 - 1) ? 0 : c + 1;
      d2 = 0.5f * (at(a, b, cq) - at(a, b, cm));
    } else if (c == 0) {
      d2 = at(a, b, 1) - at(a, b, 0);
    } else if (c == g.n2 - 1) {
      d2 = at(a, b, g.n2 - 1) - at(a, b, g.n2 - 2);
    } else {
      d2 = 0.5f * (at(a, b, c + 1) - at(a, b, c - 1));
    }
    nfg[idx] = make_float4(at(a, b, c), d0, d1, d2);
    te_out[idx] = te[((long long)a * g.n1 + b) * g.n2 + c];
  }
}

__global__ void k_validate(const float* __restrict__ ne, const float* __restrict__ te, long long n, int* bad) {
  int cnt = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float x = ne[i], t = te[i];
    if (!(isfinite(x) && x >= 0.0f && isfinite(t) && t > 0.0f)) ++cnt;
  }
  if (cnt) atomicAdd(bad, cnt);
}

// Model values from their natural logarithms: n_e = exp(ln n_e), T = exp(ln T).
__global__ void k_exp_pair(const float* __restrict__ lne, const float* __restrict__ lte, long long n,
                           float* __restrict__ ne, float* __restrict__ te) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    ne[i] = expf(lne[i]);
    te[i] = expf(lte[i]);
  }
}

__global__ void k_fill_u32(unsigned* p, unsigned v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Per-pixel launch table (shared by all frequencies and models of a call): the
// start point on the r_max sphere and its grid index in FP64 with the library
// functions, and n_e there for every model (for p0 = n(r0) (-o)).
template <int KIND>
__global__ __launch_bounds__(256) void k_launch_table(TraceArgs a, double* out, float* ne_out) {
  __shared__ float4 lds_c[4][8][kWaveLanes];
  __shared__ float lds_t[4][8][kWaveLanes];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = a.nu * a.nv;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const int i = p / a.nu, j = p - (p / a.nu) * a.nu;
    double pu, pv, b2, x0;
    pixel_start(a, i, j, pu, pv, b2, x0);
    double* L = out + size_t(p) * 6;
    if (b2 >= a.g.r_max * a.g.r_max) {
      L[0] = pu * a.u[0] + pv * a.v[0];
      L[1] = pu * a.u[1] + pv * a.v[1];
      L[2] = pu * a.u[2] + pv * a.v[2];
      L[3] = -1.0; L[4] = sqrt(b2); L[5] = 0.0;
      for (int m = 0; m < a.n_models; ++m) ne_out[size_t(m) * n + p] = 0.0f;
      continue;
    }
    RayState R;
    R.rx = x0 * a.o[0] + pu * a.u[0] + pv * a.v[0];
    R.ry = x0 * a.o[1] + pu * a.u[1] + pv * a.v[1];
    R.rz = x0 * a.o[2] + pu * a.u[2] + pv * a.v[2];
    index_exact<KIND>(a.g, R.rx, R.ry, R.rz, R.b0, R.b1, R.b2);
    if (!(R.b0 >= 0.0)) R.b0 = 0.0;  // on the sphere the radial index is the last one (>= 0)
    L[0] = R.rx; L[1] = R.ry; L[2] = R.rz; L[3] = R.b0; L[4] = R.b1; L[5] = R.b2;
    StepOrigin O;
    make_origin<KIND>(R, O);
    for (int m = 0; m < a.n_models; ++m) {
      CellCache C;
      C.key = -1;
      C.c = &lds_c[wave][0][lane];
      C.t = &lds_t[wave][0][lane];
      float ne, t;
      eval_value<KIND, true>(a.g, a.models[m].nfg, a.models[m].te, C, O, 0.f, 0.f, 0.f, ne, t);
      ne_out[size_t(m) * n + p] = ne;
    }
  }
}

// ---------------------------------------------------------------------------
// Per-wave statistics.
// ---------------------------------------------------------------------------
struct LaneStats {
  unsigned long long steps;
  unsigned max_steps;
  unsigned count[6];
};

__device__ __forceinline__ void lane_stats_add(LaneStats& s, int n, int code) {
  s.steps += (unsigned long long)n;
  s.max_steps = max(s.max_steps, (unsigned)n);
#pragma unroll
  for (int k = 0; k < 6; ++k) s.count[k] += (code == k) ? 1u : 0u;
}

__device__ void wave_stats_flush(const LaneStats& s, rt_trace_stats* out) {
  if (!out) return;
  unsigned long long st = s.steps;
  unsigned mx = s.max_steps;
  unsigned c[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) c[k] = s.count[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    st += __shfl_xor(st, off);
    mx = max(mx, (unsigned)__shfl_xor((int)mx, off));
#pragma unroll
    for (int k = 0; k < 6; ++k) c[k] += (unsigned)__shfl_xor((int)c[k], off);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&out->ray_steps, st);
    atomicMax(&out->max_steps, mx);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (c[k]) atomicAdd(&out->code_count[k], c[k]);
  }
}

// Blocks are dealt to the 8 dies round-robin; give each die a contiguous run of
// logical blocks (a band of image rows) so that its L2 sees neighbouring rays.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int x = bid % kXcds, k = bid / kXcds;
  const int per = nblocks / kXcds, rem = nblocks % kXcds;
  return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// ---------------------------------------------------------------------------
// One launch per (model, frequency) image: a wave traces one 8x8 pixel tile.
// ---------------------------------------------------------------------------
// MODE kModeCarried: the ray tube is carried along the whole ray by two
// neighbour rays (launched across the initial direction) instead of being
// retraced at every step.
template <int PREC, int KIND, int MODE = kModeFlags>
__global__ __launch_bounds__(256, MODE == kModeCarried ? 1 : 2) void k_trace_plain(TraceArgs a) {
  __shared__ float4 lds_c[4][8][kWaveLanes];
  __shared__ float lds_t[4][8][kWaveLanes];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  const int ty = tile / a.tiles_u, tx = tile - ty * a.tiles_u;
  if (ty >= a.tiles_v) return;  // whole wave
  const int j = tx * kTile + (lane & 7), i = ty * kTile + (lane >> 3);
  LaneStats st{};
  if (i < a.nv && j < a.nu) {
    typename StateOf<PREC>::type R;
    CellCache C;
    C.key = -1;
    C.c = &lds_c[wave][0][lane];
    C.t = &lds_t[wave][0][lane];
    if (init_ray(a, a.image0, i * a.nu + j, R, C)) {
      if constexpr (MODE == kModeCarried) init_tube<KIND>(a, R, C);
      int code;
      do {
        code = ray_step<PREC != kPrecFp32, KIND, MODE>(a, R, C);
      } while (code == kRunning);
      finish_ray(a, R);
      lane_stats_add(st, R.n, code);
    } else {
      lane_stats_add(st, 0, kMiss);
    }
  }
  wave_stats_flush(st, a.stats);
}

// Persistent launch over all (model, frequency, tile) work.  Tiles are split
// into kXcds ranges (one band of image rows of every image each); a wave claims
// a tile from its home range (then from the others) and hands its 64 rays to
// idle lanes in lane order.  A lane whose ray has finished takes the next ray at
// the following step, so lanes stay busy while rays of very different lengths
// finish at different times.  The loop ends when every range is exhausted and no
// lane holds a ray; each ray takes at most max_steps steps, so every wave ends.
__device__ __forceinline__ int tile_slot_ray(const TraceArgs& a, int t, int slot, int& img_out) {
  int x = 0;
  while (x < kXcds - 1 && t >= a.range_lo[x + 1]) ++x;
  const int local = t - a.range_lo[x];
  const int row0 = (x * a.tiles_v) / a.n_bands;
  const int row1 = ((x + 1) * a.tiles_v) / a.n_bands;
  const int per_image = (row1 - row0) * a.tiles_u;
  const int img = local / per_image;
  const int rem = local - img * per_image;
  const int ty = row0 + rem / a.tiles_u;
  const int tx = rem - (rem / a.tiles_u) * a.tiles_u;
  const int i = ty * kTile + (slot >> 3), j = tx * kTile + (slot & 7);
  img_out = img;
  if (i >= a.nv || j >= a.nu) return -1;
  return i * a.nu + j;
}

template <int PREC, int KIND, int MODE = kModeFlags>
__global__ __launch_bounds__(256, 2) void k_trace_persistent(TraceArgs a) {
  __shared__ float4 lds_c[4][8][kWaveLanes];
  __shared__ float lds_t[4][8][kWaveLanes];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int home = blockIdx.x % kXcds;
  unsigned exhausted = 0;
  int pool_left = 0, cur_tile = -1;
  bool active = false;
  typename StateOf<PREC>::type R;
  CellCache C;
  C.key = -1;
  C.c = &lds_c[wave][0][lane];
  C.t = &lds_t[wave][0][lane];
  // statistics: per-lane step sum and maximum; rays per code counted by ballot
  unsigned long long lane_steps = 0;
  unsigned lane_max = 0;
  unsigned code_cnt[6] = {0, 0, 0, 0, 0, 0};
  const unsigned all = (1u << kXcds) - 1u;
  for (;;) {
    unsigned long long idle = __ballot(!active);
    // refill once enough lanes are idle (or none is busy): fewer, larger refills keep
    // the lanes of a wave at similar depths along their rays
    if (__popcll(idle) < a.refill_min_idle && idle != ~0ull) idle = 0ull;
    while (idle != 0ull && (pool_left > 0 || exhausted != all)) {
      if (pool_left == 0) {
        int t = -1;
        for (int k = 0; k < kXcds && t < 0; ++k) {
          const int x = (home + k) % kXcds;
          if (exhausted & (1u << x)) continue;
          unsigned got = 0;
          if (lane == 0) got = atomicAdd(&a.counters[x], 1u);
          got = (unsigned)__shfl((int)got, 0);
          const int len = a.range_lo[x + 1] - a.range_lo[x];
          if ((int)got < len) t = a.range_lo[x] + (int)got;
          else exhausted |= 1u << x;
        }
        if (t < 0) break;
        cur_tile = t;
        pool_left = 64;
      }
      const int rank = __popcll(idle & ((1ull << lane) - 1ull));
      const int take = min(__popcll(idle), pool_left);
      bool missed = false;
      if (!active && rank < take) {
        int img;
        const int pix = tile_slot_ray(a, cur_tile, (64 - pool_left) + rank, img);
        if (pix >= 0) {
          if (init_ray(a, img, pix, R, C)) active = true;
          else missed = true;
        }
      }
      code_cnt[kMiss] += (unsigned)__popcll(__ballot(missed));
      pool_left -= take;
      idle = __ballot(!active);
    }
    if (__ballot(active) == 0ull) break;
    int done = kRunning;
    if (active) {
      const int code = ray_step<PREC != kPrecFp32, KIND, MODE>(a, R, C);
      if (code != kRunning) {
        finish_ray(a, R);
        active = false;
        lane_steps += (unsigned long long)R.n;
        lane_max = max(lane_max, (unsigned)R.n);
        done = code;
      }
    }
    if (__ballot(done != kRunning)) {
#pragma unroll
      for (int k = 1; k < 6; ++k)
        if (k != kMiss) code_cnt[k] += (unsigned)__popcll(__ballot(done == k));
    }
  }
  LaneStats st{};
  st.steps = lane_steps;
  st.max_steps = lane_max;
  if (lane == 0)
    for (int k = 0; k < 6; ++k) st.count[k] = code_cnt[k];
  wave_stats_flush(st, a.stats);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static int grid_for(long long n, int threads) {
  long long b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return int(b);
}

hipError_t launch_pack(const DevGeom& g, const float* ne, const float* te, float4* nfg, float* te_out, hipStream_t s) {
  const long long total = (long long)g.n0 * g.n1 * g.n2p;
  hipLaunchKernelGGL(k_pack, dim3(grid_for(total, 256)), dim3(256), 0, s, g, ne, te, nfg, te_out);
  return hipGetLastError();
}

hipError_t launch_validate(const float* ne, const float* te, long long n, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n, 256)), dim3(256), 0, s, ne, te, n, bad);
  return hipGetLastError();
}

hipError_t launch_exp_pair(const float* lne, const float* lte, long long n, float* ne, float* te, hipStream_t s) {
  hipLaunchKernelGGL(k_exp_pair, dim3(grid_for(n, 256)), dim3(256), 0, s, lne, lte, n, ne, te);
  return hipGetLastError();
}

hipError_t launch_start_index(const TraceArgs& a, double* out, float* ne_out, hipStream_t s) {
  const long long n = (long long)a.nu * a.nv;
  if (a.g.kind == RT_GRID_SPHERICAL_LOGR)
    hipLaunchKernelGGL((k_launch_table<RT_GRID_SPHERICAL_LOGR>), dim3(grid_for(n, 256)), dim3(256), 0, s, a, out, ne_out);
  else
    hipLaunchKernelGGL((k_launch_table<RT_GRID_CARTESIAN>), dim3(grid_for(n, 256)), dim3(256), 0, s, a, out, ne_out);
  return hipGetLastError();
}

// Number of 32-bit words that differ between a and b (added to *count).
__global__ void k_count_diff(const unsigned* a, const unsigned* b, long long n, unsigned* count) {
  unsigned c = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    c += (a[i] != b[i]) ? 1u : 0u;
  if (c) atomicAdd(count, c);
}

hipError_t launch_count_diff(const unsigned* a, const unsigned* b, long long n, unsigned* count, hipStream_t s) {
  hipLaunchKernelGGL(k_count_diff, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n, count);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, unsigned val, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, val, n);
  return hipGetLastError();
}

// The two reduced tracing modes (line of sight; refraction without the tube
// term) are fixed at compile time for the default-precision kernels: without
// the perturbed retraces the step needs far fewer registers and these kernels
// run at 3-4 waves per SIMD.  The full method keeps the mode in the call's flags
// (its compile-time instance spills more and is slower: 993 ms against 979 ms
// on the structured stack), and so do the FP32-stepping and all-FP32 variants.
static int launch_mode(int prec, uint32_t flags) {
  if (prec != kPrecDefault) return kModeFlags;
  if (!(flags & RT_USE_REFRACTION)) return kModeLos;
  return (flags & RT_USE_MAGNIFICATION) ? kModeFlags : kModeNoMag;
}

template <int PREC, int KIND, int MODE>
static hipError_t launch_in_mode(const TraceArgs& a, bool plain, int blocks, hipStream_t s) {
  if (plain) hipLaunchKernelGGL((k_trace_plain<PREC, KIND, MODE>), dim3(blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_trace_persistent<PREC, KIND, MODE>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int KIND>
static hipError_t launch_kind(const TraceArgs& a, bool plain, int prec, int blocks, hipStream_t s) {
  if (a.flags & RT_CARRIED_TUBE) {
    // carried tubes: default precision, one launch per image
    if (prec != kPrecDefault || !plain) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_trace_plain<kPrecDefault, KIND, kModeCarried>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (prec == kPrecFp32) return launch_in_mode<kPrecFp32, KIND, kModeFlags>(a, plain, blocks, s);
  if (prec == kPrecFp32Step) return launch_in_mode<kPrecFp32Step, KIND, kModeFlags>(a, plain, blocks, s);
  switch (launch_mode(prec, a.flags)) {
    case kModeLos: return launch_in_mode<kPrecDefault, KIND, kModeLos>(a, plain, blocks, s);
    case kModeNoMag: return launch_in_mode<kPrecDefault, KIND, kModeNoMag>(a, plain, blocks, s);
    default: return launch_in_mode<kPrecDefault, KIND, kModeFlags>(a, plain, blocks, s);
  }
}

hipError_t launch_trace(const TraceArgs& a, bool plain, int prec, int blocks, hipStream_t s) {
  if (a.g.kind == RT_GRID_SPHERICAL_LOGR) return launch_kind<RT_GRID_SPHERICAL_LOGR>(a, plain, prec, blocks, s);
  return launch_kind<RT_GRID_CARTESIAN>(a, plain, prec, blocks, s);
}

template <int PREC, int KIND, int MODE>
static hipError_t occupancy_of(int* n) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_trace_persistent<PREC, KIND, MODE>, 256, 0);
}

template <int KIND>
static hipError_t occupancy_kind(int* n, int prec, uint32_t flags) {
  if (prec == kPrecFp32) return occupancy_of<kPrecFp32, KIND, kModeFlags>(n);
  if (prec == kPrecFp32Step) return occupancy_of<kPrecFp32Step, KIND, kModeFlags>(n);
  switch (launch_mode(prec, flags)) {
    case kModeLos: return occupancy_of<kPrecDefault, KIND, kModeLos>(n);
    case kModeNoMag: return occupancy_of<kPrecDefault, KIND, kModeNoMag>(n);
    default: return occupancy_of<kPrecDefault, KIND, kModeFlags>(n);
  }
}

int persistent_blocks_per_cu(int prec, int kind, uint32_t flags) {
  int n = 0;
  const hipError_t e = kind == RT_GRID_SPHERICAL_LOGR ? occupancy_kind<RT_GRID_SPHERICAL_LOGR>(&n, prec, flags)
                                                      : occupancy_kind<RT_GRID_CARTESIAN>(&n, prec, flags);
  if (e != hipSuccess || n < 1) n = 1;
  return n;
}

}  // namespace rt
