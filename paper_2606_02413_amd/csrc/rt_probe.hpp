// Launcher of the streaming-read probe (rt_probe.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "rt_internal.hpp"

namespace rt {

// span4 <= n4, blocks >= 1; sink holds blocks x 256 floats (written only for a
// buffer that is not zero-filled)
hipError_t launch_stream_read(const float4* buf, long long n4, long long span4, int blocks, int reps, float* sink,
                              hipStream_t s);

// path: [n_walks][cap][kPathStride] records of the tracer, path_len [n_walks];
// keys: [cap][n_walks]
hipError_t launch_path_keys(const DevGeom& g, const float* path, const int* path_len, int n_walks, int cap, int* keys,
                            hipStream_t s);

// keys: [cap][n_walks]; sink: n_walks floats (written only where a walk's sum
// happens to equal 12345.5; in bounds either way)
hipError_t launch_gather_replay(const float4* nfg, const float* te, const int* keys, int n_walks, int cap, int s0,
                                int s1, int max_key, float* sink, hipStream_t s);

}  // namespace rt
