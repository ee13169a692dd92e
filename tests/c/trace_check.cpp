// A trace through the C ABI with no Python in between: loads a model from two
// float32 files (C-order [n0][n1][n2] n_e and T of a spherical log-r grid),
// traces one image at the given frequencies with the library's defaults, and
// writes the T_b maps [freq][nv][nu] (float32) and the per-ray step counts
// (int32) to files.
//   trace_check N0 N1 N2 R_IN R_MAX NE_FILE TE_FILE NPIX HALF OUT_TB OUT_STEPS F1 [F2 ...]
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rtsun.h"

static bool read_all(const char* path, std::vector<float>& v) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  const size_t got = std::fread(v.data(), sizeof(float), v.size(), f);
  std::fclose(f);
  return got == v.size();
}

static int fail(const char* what, rt_status s) {
  std::printf("%s: %s (%s)\n", what, rt_status_string(s), rt_last_error_message());
  return 1;
}

int main(int argc, char** argv) {
  if (argc < 13) {
    std::printf("usage: trace_check N0 N1 N2 R_IN R_MAX NE TE NPIX HALF OUT_TB OUT_STEPS F1 [F2 ...]\n");
    return 2;
  }
  rt_grid_desc d = {};
  d.abi_version = RT_ABI_VERSION;
  d.kind = RT_GRID_SPHERICAL_LOGR;
  d.n0 = std::atoi(argv[1]); d.n1 = std::atoi(argv[2]); d.n2 = std::atoi(argv[3]);
  d.r_in = std::atof(argv[4]); d.r_max = std::atof(argv[5]);
  const size_t nv = size_t(d.n0) * d.n1 * d.n2;
  std::vector<float> ne(nv), te(nv);
  if (!read_all(argv[6], ne) || !read_all(argv[7], te)) { std::printf("cannot read the model\n"); return 1; }
  const int npix = std::atoi(argv[8]);
  const double half = std::atof(argv[9]);
  std::vector<double> freqs;
  for (int k = 12; k < argc; ++k) freqs.push_back(std::atof(argv[k]));
  const int nf = int(freqs.size());

  rt_model* m = nullptr;
  rt_status s = rt_model_load(&d, ne.data(), te.data(), 0, nullptr, &m);
  if (s != RT_OK) return fail("rt_model_load", s);
  rt_image_desc im = {};
  im.obs_dir[0] = 1.0; im.up[2] = 1.0; im.nu = npix; im.nv = npix; im.half_u = half; im.half_v = half;
  rt_params p;
  rt_params_default(&p);
  const size_t n_rays = size_t(nf) * npix * npix;
  float* tb = nullptr;
  rt_ray_info* info = nullptr;
  if (hipMalloc(&tb, n_rays * sizeof(float)) != hipSuccess ||
      hipMalloc(&info, n_rays * sizeof(rt_ray_info)) != hipSuccess) {
    std::printf("hipMalloc failed\n");
    return 1;
  }
  const rt_model* models[1] = {m};
  s = rt_trace_maps(models, 1, freqs.data(), nf, &im, &p, tb, info, nullptr, nullptr, 0, 0, nullptr, nullptr,
                    nullptr);
  if (s != RT_OK) return fail("rt_trace_maps", s);
  std::vector<float> h_tb(n_rays);
  std::vector<rt_ray_info> h_info(n_rays);
  if (hipMemcpy(h_tb.data(), tb, n_rays * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(h_info.data(), info, n_rays * sizeof(rt_ray_info), hipMemcpyDeviceToHost) != hipSuccess) {
    std::printf("copy back failed\n");
    return 1;
  }
  std::vector<int> steps(n_rays);
  for (size_t i = 0; i < n_rays; ++i) steps[i] = h_info[i].n_steps;
  FILE* f = std::fopen(argv[10], "wb");
  FILE* g = std::fopen(argv[11], "wb");
  if (!f || !g) { std::printf("cannot write the outputs\n"); return 1; }
  std::fwrite(h_tb.data(), sizeof(float), n_rays, f);
  std::fwrite(steps.data(), sizeof(int), n_rays, g);
  std::fclose(f);
  std::fclose(g);
  (void)hipFree(tb);
  (void)hipFree(info);
  rt_model_free(m);
  std::printf("ok %zu rays\n", n_rays);
  return 0;
}
