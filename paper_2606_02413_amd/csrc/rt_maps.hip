// Post-processing of brightness-temperature maps: convolution with a Gaussian
// interferometric beam (the synthetic maps of Sec. 3.3 are shown convolved),
// and the mean T_b of the disc centre at each frequency (the brightness-
// temperature spectrum of Sec. 3.4.1).
#include <hip/hip_runtime.h>

#include "rt_internal.hpp"

namespace rt {

// One pass of the separable beam along u (ALONG_U) or v of every map: out =
// sum_k w_k in[. + k], w_k = exp(-k^2 / (2 sigma^2)) / norm for |k| <= radius,
// zero outside the image (the sky around the image is dark).  One thread per
// output pixel; the taps are read through L1/L2.
template <bool ALONG_U>
__global__ void k_blur(BlurArgs b, const float* __restrict__ in, float* __restrict__ out) {
  const long long per_map = (long long)b.nu * b.nv;
  const long long total = per_map * b.n_maps;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int m = int(q / per_map);
    const long long pix = q - m * per_map;
    const int i = int(pix / b.nu), j = int(pix - (long long)i * b.nu);
    const int R = ALONG_U ? b.radius_u[m] : b.radius_v[m];
    const float c = ALONG_U ? b.inv2s2_u[m] : b.inv2s2_v[m];
    const float inv_norm = ALONG_U ? b.inv_norm_u[m] : b.inv_norm_v[m];
    const int pos = ALONG_U ? j : i, len = ALONG_U ? b.nu : b.nv;
    const long long stride = ALONG_U ? 1 : b.nu;
    const float* row = in + m * per_map + pix - (long long)pos * stride;
    const int k0 = max(-R, -pos), k1 = min(R, len - 1 - pos);
    float acc = 0.0f;
    for (int k = k0; k <= k1; ++k) acc = fmaf(__expf(-float(k * k) * c), row[(long long)(pos + k) * stride], acc);
    out[q] = acc * inv_norm;
  }
}

// Mean of each map over the pixels whose centre lies within `radius` of the
// image centre: one block per map, FP64 sums reduced in LDS.
__global__ __launch_bounds__(256) void k_disc_mean(DiscArgs d, const float* __restrict__ maps,
                                                   double* __restrict__ out) {
  __shared__ double s_sum[256];
  __shared__ double s_cnt[256];
  const int m = blockIdx.x;
  const long long per_map = (long long)d.nu * d.nv;
  const float* map = maps + m * per_map;
  double sum = 0.0, cnt = 0.0;
  for (long long p = threadIdx.x; p < per_map; p += blockDim.x) {
    const int i = int(p / d.nu), j = int(p - (long long)i * d.nu);
    const double u = -d.half_u + (j + 0.5) * d.pix_u, v = -d.half_v + (i + 0.5) * d.pix_v;
    if (u * u + v * v < d.radius2) {
      sum += double(map[p]);
      cnt += 1.0;
    }
  }
  s_sum[threadIdx.x] = sum;
  s_cnt[threadIdx.x] = cnt;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = s_cnt[0] > 0.0 ? s_sum[0] / s_cnt[0] : 0.0;
}

static int grid_for_maps(long long n) {
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return int(b);
}

hipError_t launch_blur(const BlurArgs& b, const float* in, float* tmp, float* out, hipStream_t s) {
  const long long total = (long long)b.nu * b.nv * b.n_maps;
  hipLaunchKernelGGL(k_blur<true>, dim3(grid_for_maps(total)), dim3(256), 0, s, b, in, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_blur<false>, dim3(grid_for_maps(total)), dim3(256), 0, s, b, tmp, out);
  return hipGetLastError();
}

hipError_t launch_disc_mean(const DiscArgs& d, const float* maps, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_disc_mean, dim3(d.n_maps), dim3(256), 0, s, d, maps, out);
  return hipGetLastError();
}

}  // namespace rt
