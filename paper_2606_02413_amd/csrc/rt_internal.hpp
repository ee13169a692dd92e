// Internal declarations shared by the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rtsun.h"

namespace rt {

constexpr int kMaxModels = 16;    // models per persistent launch
constexpr int kMaxFreqs = 128;    // frequencies per persistent launch
constexpr int kTile = 8;          // 8 x 8 pixels per wave64
constexpr int kWaveLanes = 64;
constexpr int kXcds = 8;          // MI355X: 8 accelerator complex dies, blocks dealt round-robin
constexpr int kPathStride = 9;    // x y z s lnM dlnS/ds tau ne te

// Grid geometry common to every model of a call.
struct DevGeom {
  int kind;             // rt_grid_kind
  int n0, n1, n2, n2p;  // n2p: row length of the packed arrays (n2 + 1 for the periodic phi axis)
  float ln_rin, inv_dl, inv_dth, inv_dph;  // spherical
  float org[3], inv_sp[3];                 // Cartesian
  double ln_rin_d, inv_dl_d, inv_dth_d, inv_dph_d;
  double org_d[3], inv_sp_d[3];
  double r_in, r_max;
  int has_inner;
};

struct DevModelPtrs {
  const float4* nfg;    // per vertex: n_e, dn/dxi_0, dn/dxi_1, dn/dxi_2 (index-space gradient)
  const float* te;      // per vertex: T
};

struct TraceArgs {
  DevGeom g;
  DevModelPtrs models[kMaxModels];
  double freqs[kMaxFreqs];
  double xf[kMaxFreqs];       // X / n_e = (8.98e3 / f)^2 per frequency
  float lnf[kMaxFreqs];       // ln f per frequency
  const double* launch;       // [nv * nu][6]: start point r0 and its continuous grid index
                              // (missing pixels: their image-plane point, index0 = -1, index1 = b)
  const float* launch_ne;     // [n_models][nv * nu]: n_e at each pixel's start point
  int n_models, n_freq;
  int nu, nv, tiles_u, tiles_v, tiles_per_image;
  int image0;                 // plain launches: flat (model * n_freq + freq) index of the image
  double o[3], u[3], v[3];    // observer axes
  double half_u, half_v;
  float ds_max, n_floor, eta;
  double ds_max_d, n_floor_d;
  int max_steps;
  double tb_inner, tb_sky;
  uint32_t flags;
  float* tb;
  rt_ray_info* info;
  rt_trace_stats* stats;
  const int32_t* path_rays;
  int n_path, path_cap;
  float* path_out;
  int32_t* path_len;
  // persistent scheduling: tiles are split into kXcds contiguous ranges
  unsigned* counters;         // kXcds claim counters (zeroed before launch)
  int range_lo[kXcds + 1];
  int n_bands;                // image rows split into bands, one per range
  int refill_min_idle;        // a wave refills once at least this many lanes are idle (1..64)
};

// Reverse-mode (adjoint) launches over one model, per batch of tiles: the
// forward trace of every ray with checkpoints, then the reverse sweeps.
constexpr int kCkptFields = 10;   // r (3), p (3), grid index (3), optical depth so far
constexpr int kGradChannels = 5;  // per vertex: n_e, the three index-space gradient channels, T
// Per-step record of the forward quantities the reverse sweep needs (FP32):
// n(r_i), F1, F2, sum g1+g2+g3, g1+2g2+2g3+g4, q1 and the force-difference sums
// of the two perturbed retraces, n_e and T at the chord midpoint.
enum : int {
  kTapeNi = 0, kTapeF1 = 1, kTapeF2 = 4, kTapeS = 7, kTapeT = 10, kTapeQ = 13, kTapeA = 19,
  kTapeNeM = 25, kTapeTeM = 26, kTapeFields = 27
};
struct AdjointArgs {
  TraceArgs t;                // one model, image layout [freq][nv][nu]
  const float* weights;       // [n_freq][nv][nu]
  double* loss;               // device scalar, accumulated
  double* gacc;               // [n0 * n1 * n2p][kGradChannels] channel adjoints, zeroed before launch
  double* ckpt;               // [ckpt_cap][kCkptFields][n_rays] checkpoints of the batch's rays
  int* meta;                  // [3][n_rays] per ray: steps to sweep (0: none), code | checkpoints << 8, interval
  double* steps;              // [K][kCkptFields][n_slots] start state of each step of a chunk
  float* tape;                // [K][kTapeFields][n_slots] forward record of each step of a chunk
  unsigned* counter;          // tile claim counter of the sweep, zeroed before launch
  int K, ckpt_cap, n_slots;
  int tile0, n_tiles;         // the batch: tiles tile0 .. tile0 + n_tiles - 1 (8x8 pixels of one frequency)
  int n_rays;                 // 64 n_tiles; ray rid = 64 (tile - tile0) + lane
};

// Map post-processing (rt_maps.hip).
constexpr int kMaxBlurMaps = 128;   // maps per beam-convolution call
struct BlurArgs {
  int n_maps, nu, nv;
  int radius_u[kMaxBlurMaps], radius_v[kMaxBlurMaps];          // taps |k| <= radius
  float inv2s2_u[kMaxBlurMaps], inv2s2_v[kMaxBlurMaps];        // 1 / (2 sigma^2), sigma in pixels
  float inv_norm_u[kMaxBlurMaps], inv_norm_v[kMaxBlurMaps];    // 1 / sum of the taps
};
struct DiscArgs {
  int n_maps, nu, nv;
  double half_u, half_v, pix_u, pix_v, radius2;
};
hipError_t launch_blur(const BlurArgs& b, const float* in, float* tmp, float* out, hipStream_t s);
hipError_t launch_disc_mean(const DiscArgs& d, const float* maps, double* out, hipStream_t s);

// Launchers (rt_kernels.hip).
hipError_t launch_pack(const DevGeom& g, const float* ne, const float* te, float4* nfg, float* te_out,
                       hipStream_t s);
hipError_t launch_validate(const float* ne, const float* te, long long n, int* bad, hipStream_t s);
hipError_t launch_exp_pair(const float* lne, const float* lte, long long n, float* ne, float* te, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, unsigned val, long long n, hipStream_t s);
hipError_t launch_count_diff(const unsigned* a, const unsigned* b, long long n, unsigned* count, hipStream_t s);
// prec: kPrecDefault, kPrecFp32Step or kPrecFp32 (rt_trace.hpp), from precision_of(flags)
hipError_t launch_trace(const TraceArgs& a, bool plain, int prec, int grid_blocks, hipStream_t s);
hipError_t launch_start_index(const TraceArgs& a, double* out, float* ne_out, hipStream_t s);
int persistent_blocks_per_cu(int prec, int kind, uint32_t flags);
inline int precision_of(uint32_t flags) {
  return (flags & RT_PREC_ALL_FP32) ? 2 : (flags & RT_PREC_FP32_STEP) ? 1 : 0;
}

// Launchers (rt_adjoint.hip).
hipError_t launch_adjoint_forward(const AdjointArgs& a, hipStream_t s);
hipError_t launch_adjoint(const AdjointArgs& a, int blocks, hipStream_t s);
hipError_t launch_unpack_grad(const DevGeom& g, const float4* nfg, const float* te, const double* gacc,
                              float* grad_ln_ne, float* grad_ln_te, hipStream_t s);
int adjoint_blocks_per_cu(int kind);

}  // namespace rt

static_assert(sizeof(rt_ray_info) == 32, "rt_ray_info is 32 bytes");
static_assert(sizeof(rt_trace_stats) == 40, "rt_trace_stats is 40 bytes");
static_assert(sizeof(rt::AdjointArgs) <= 4096, "kernel arguments fit the 4 KiB argument segment");
static_assert(sizeof(rt::BlurArgs) <= 4096, "kernel arguments fit the 4 KiB argument segment");
