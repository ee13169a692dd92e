// Launcher of the streaming-read probe (rt_probe.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace rt {

// span4 <= n4, blocks >= 1; sink holds blocks x 256 floats (written only for a
// buffer that is not zero-filled)
hipError_t launch_stream_read(const float4* buf, long long n4, long long span4, int blocks, int reps, float* sink,
                              hipStream_t s);

}  // namespace rt
