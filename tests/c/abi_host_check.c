/* The C ABI used from plain C99 (no Python, no device work): constants,
 * defaults, status strings and the host-side validation of every class of
 * argument error.  Prints "ok" and exits 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "rtsun.h"

static int fails = 0;
#define CHECK(c)                                            \
  do {                                                      \
    if (!(c)) {                                             \
      printf("check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                              \
    }                                                       \
  } while (0)

int main(void) {
  CHECK(sizeof(rt_ray_info) == 32);
  CHECK(sizeof(rt_trace_stats) == 40);
  CHECK(rt_abi_version() == RT_ABI_VERSION);

  rt_params p;
  rt_params_default(&p);
  CHECK(p.abi_version == RT_ABI_VERSION);
  CHECK(p.flags == (RT_USE_MAGNIFICATION | RT_USE_REFRACTION));
  CHECK(p.ds_max == 0.005 && p.n_floor == 1.0 && p.max_steps == 200000 && p.checkpoint_every == 64);
  rt_tuning t;
  rt_tuning_default(&t);
  CHECK(t.refill_min_idle == 64 && t.blocks_per_cu == 0 && t.xcd_bands == 8);
  CHECK(strcmp(rt_status_string(RT_E_CAPACITY), "RT_E_CAPACITY") == 0);

  /* model descriptors: refused before any value or device is touched */
  float ne[8] = {1e7f, 1e7f, 1e7f, 1e7f, 1e7f, 1e7f, 1e7f, 1e7f};
  float te[8] = {1e6f, 1e6f, 1e6f, 1e6f, 1e6f, 1e6f, 1e6f, 1e6f};
  rt_model* m = NULL;
  CHECK(rt_model_load(NULL, ne, te, 0, NULL, &m) == RT_E_INVALID_ARG && m == NULL);
  CHECK(strlen(rt_last_error_message()) > 0);
  rt_grid_desc d;
  memset(&d, 0, sizeof d);
  d.abi_version = RT_ABI_VERSION;
  d.kind = RT_GRID_SPHERICAL_LOGR;
  d.n0 = 4096; d.n1 = 4096; d.n2 = 3;  /* n0 * n1 = 2^24: beyond the cell-key range */
  d.r_in = 1.0; d.r_max = 3.0;
  CHECK(rt_model_load(&d, ne, te, 0, NULL, &m) == RT_E_CAPACITY && m == NULL);
  d.n0 = 2; d.n1 = 2; d.n2 = 2;  /* spherical grids need n2 >= 3 */
  CHECK(rt_model_load(&d, ne, te, 0, NULL, &m) == RT_E_INVALID_ARG);
  d.abi_version = 99;
  CHECK(rt_model_load(&d, ne, te, 0, NULL, &m) == RT_E_INVALID_ARG);

  /* trace calls: argument errors */
  double f = 150e6;
  rt_image_desc im;
  memset(&im, 0, sizeof im);
  im.obs_dir[0] = 1.0; im.up[2] = 1.0; im.nu = 8; im.nv = 8; im.half_u = 2.0; im.half_v = 2.0;
  CHECK(rt_trace_maps(NULL, 0, &f, 1, &im, &p, NULL, NULL, NULL, NULL, 0, 0, NULL, NULL, NULL) ==
        RT_E_INVALID_ARG);

  /* beam widths (host arithmetic of the ABI): lambda / B as an angle, in R_sun at 1 au */
  double fw[2], fq[2] = {100e6, 300e6};
  CHECK(rt_beam_fwhm(fq, 2, 5e3, fw) == RT_OK);
  const double want = 299792458.0 / 100e6 / 5e3 / (6.957e8 / 1.495978707e11);
  CHECK(fabs(fw[0] / want - 1.0) < 1e-15 && fabs(fw[0] / fw[1] - 3.0) < 1e-14);
  CHECK(rt_beam_fwhm(fq, 2, 0.0, fw) == RT_E_INVALID_ARG);

  if (fails) return 1;
  printf("ok\n");
  return 0;
}
