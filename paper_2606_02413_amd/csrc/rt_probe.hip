// Measurement probe: streaming float4 reads of a device buffer, for the
// bandwidth figures the tracer is compared with (the die-local L2, the
// Infinity Cache and HBM).  Not part of the method.
#include <hip/hip_runtime.h>

#include "rt_probe.hpp"

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

}  // namespace rt
