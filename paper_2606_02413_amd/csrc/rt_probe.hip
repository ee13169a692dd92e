// Measurement probes, not part of the method: streaming float4 reads of a
// device buffer (the bandwidth of the die-local L2, the Infinity Cache and
// HBM), and a gather-only replay of the tracer's recorded cell walks (the rate
// at which the memory system serves the tracer's gathers without its
// arithmetic).
#include <hip/hip_runtime.h>

#include "rt_probe.hpp"
#include "rt_trace.hpp"

namespace rt {

// Block b reads span4 float4 of buf (n4 of them) starting at start(b), wrapping
// at the end, `reps` times.  Whole-buffer reads (span4 == n4) start each block at
// a different offset so that the blocks do not walk the channels in lock step.
// The sum is stored only if it equals a value a zero-filled buffer cannot give,
// which keeps the loads without writing anything.
__global__ __launch_bounds__(256) void k_stream_read(const float4* __restrict__ buf, long long n4, long long span4,
                                                     int reps, float* __restrict__ sink) {
  const long long start = (span4 == n4) ? ((long long)blockIdx.x * 62528) % n4 : ((long long)blockIdx.x * span4) % n4;
  float ax = 0.f, ay = 0.f, az = 0.f, aw = 0.f;
  for (int r = 0; r < reps; ++r) {
    for (long long i = threadIdx.x; i < span4; i += blockDim.x) {
      long long j = start + i;
      if (j >= n4) j -= n4;
      const float4 v = buf[j];
      ax += v.x; ay += v.y; az += v.z; aw += v.w;
    }
  }
  const float s = (ax + ay) + (az + aw);
  if (s == 12345.5f) sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

hipError_t launch_stream_read(const float4* buf, long long n4, long long span4, int blocks, int reps, float* sink,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, s, buf, n4, span4, reps, sink);
  return hipGetLastError();
}

// Cell keys of recorded path points: for record s of walk w (the point after
// step s), the tracer's key (a n1 + b) n2p + c of the cell that holds it, with
// the tracer's clamping of the r/theta (and Cartesian) cells and the periodic
// phi cell; -1 past the walk's recorded length.  keys: [cap][n_walks].
template <int KIND>
__global__ __launch_bounds__(256) void k_path_keys(DevGeom g, const float* __restrict__ path,
                                                   const int* __restrict__ path_len, int n_walks, int cap,
                                                   int* __restrict__ keys) {
  const long long total = (long long)n_walks * cap;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int s = int(q / n_walks), w = int(q - (long long)s * n_walks);
    int key = -1;
    if (s < path_len[w]) {
      const float* p = path + ((size_t)w * cap + s) * kPathStride;
      double b0, b1, b2;
      index_exact<KIND>(g, double(p[0]), double(p[1]), double(p[2]), b0, b1, b2);
      auto clamp_cell = [](double b, int n) {
        double f = floor(b);
        if (!(f >= 0.0)) f = 0.0;  // also NaN
        if (f > double(n - 2)) f = double(n - 2);
        return int(f);
      };
      const int a = clamp_cell(b0, g.n0), b = clamp_cell(b1, g.n1);
      int c;
      if constexpr (KIND == RT_GRID_SPHERICAL_LOGR) {
        double f = floor(b2);
        if (!(f >= 0.0 && f < double(g.n2))) f = 0.0;
        c = int(f);
      } else {
        c = clamp_cell(b2, g.n2);
      }
      key = (a * g.n1 + b) * g.n2p + c;
    }
    keys[q] = key;
  }
}

// Gather-only replay of recorded cell walks with the tracer's model layout and
// per-lane cell cache: lane w walks keys[.][w]; when the key changes it gathers
// the cell's 8 corners (float4 n_e and index gradient, float T) into its LDS
// slots, and every step it reads them back, as the tracer's evaluations do.
// No ray arithmetic.  A key outside [0, max_key] ends the walk (every corner
// of a key <= max_key lies inside the packed grid).
__global__ __launch_bounds__(256) void k_gather_replay(const float4* __restrict__ nfg, const float* __restrict__ te,
                                                       const int* __restrict__ keys, int n_walks, int cap, int s0,
                                                       int s1, int max_key, float* __restrict__ sink) {
  __shared__ float4 lc[8][256];
  __shared__ float lt[8][256];
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_walks) return;  // no block-wide barrier below
  const int t = threadIdx.x;
  int cached = -1;
  float acc = 0.f;
  for (int s = 0; s < cap; ++s) {
    const int key = keys[(size_t)s * n_walks + w];
    if (key < 0 || key > max_key) break;
    if (key != cached) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int off = ((k & 4) ? s0 : 0) + ((k & 2) ? s1 : 0) + (k & 1);
        lc[k][t] = nfg[key + off];
        lt[k][t] = te[key + off];
      }
      cached = key;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float4 v = lc[k][t];
      acc += (v.x + v.y) + (v.z + v.w) + lt[k][t];
    }
  }
  if (acc == 12345.5f) sink[w] = acc;
}

hipError_t launch_path_keys(const DevGeom& g, const float* path, const int* path_len, int n_walks, int cap, int* keys,
                            hipStream_t s) {
  long long total = (long long)n_walks * cap;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (g.kind == RT_GRID_SPHERICAL_LOGR)
    hipLaunchKernelGGL(k_path_keys<RT_GRID_SPHERICAL_LOGR>, dim3(int(blocks)), dim3(256), 0, s, g, path, path_len,
                       n_walks, cap, keys);
  else
    hipLaunchKernelGGL(k_path_keys<RT_GRID_CARTESIAN>, dim3(int(blocks)), dim3(256), 0, s, g, path, path_len, n_walks,
                       cap, keys);
  return hipGetLastError();
}

hipError_t launch_gather_replay(const float4* nfg, const float* te, const int* keys, int n_walks, int cap, int s0,
                                int s1, int max_key, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_replay, dim3((n_walks + 255) / 256), dim3(256), 0, s, nfg, te, keys, n_walks, cap, s0, s1,
                     max_key, sink);
  return hipGetLastError();
}

}  // namespace rt
