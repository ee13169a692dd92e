// Memory and undefined-behaviour check of the oracle (test infrastructure):
// compiled together with rt_oracle.cpp under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py, it calls every
// entry point of the oracle once on small inputs (both grids, both steppers,
// the carried tube, paths, the twin check, dual numbers and tapes) and prints
// "ok".  It sets up inputs only; all arithmetic of the method is the oracle's.
#include <cstdio>
#include <cmath>
#include <vector>

#include "rt_oracle.cpp"

namespace {

// A smooth positive field with a deterministic ripple: n_e falling with radius,
// T between 1 and 2 MK.
void fill_spherical(int nr, int nt, int np, double r_in, double r_max, std::vector<float>& ne,
                    std::vector<float>& te) {
  ne.resize(size_t(nr) * nt * np);
  te.resize(ne.size());
  unsigned s = 12345u;
  for (int a = 0; a < nr; ++a)
    for (int b = 0; b < nt; ++b)
      for (int c = 0; c < np; ++c) {
        const double r = r_in * std::pow(r_max / r_in, double(a) / (nr - 1));
        s = s * 1664525u + 1013904223u;
        const double ripple = 1.0 + 0.2 * (double(s >> 8) / double(1u << 24) - 0.5);
        const size_t i = (size_t(a) * nt + b) * np + c;
        ne[i] = float(3e8 * std::pow(r, -6.0) * ripple + 1e6);
        te[i] = float(1.0e6 + 1.0e6 * double(b) / nt);
      }
}

}  // namespace

int main() {
  using namespace orc;
  int fails = 0;
  std::vector<float> ne, te;
  fill_spherical(16, 8, 16, 1.0, 4.0, ne, te);
  Medium m{};
  m.kind = GRID_SPHERICAL_LOGR;
  m.n0 = 16; m.n1 = 8; m.n2 = 16;
  m.r_in = 1.0; m.r_max = 4.0;
  m.ne = ne.data(); m.te = te.data();
  Params P{};
  P.stepper = 0; P.use_refraction = 1; P.use_magnification = 1; P.no_absorption = 0;
  P.ds_max = 0.02; P.n_floor = 0.1; P.max_steps = 20000; P.twin_check = 1; P.eta = 1e-2;
  P.tb_inner = 1e4; P.tb_sky = 0.0; P.dp_rtol = 1e-10; P.dp_atol = 1e-10; P.carried_tube = 0;
  P.twin_exit_tol = 5e-5;
  Image im{};
  im.obs_dir[0] = 1.0; im.up[2] = 1.0;
  im.nu = 8; im.nv = 8; im.half_u = 4.5; im.half_v = 4.5;  // corners miss the model
  std::vector<int32_t> pix(64);
  for (int i = 0; i < 64; ++i) pix[size_t(i)] = i;
  std::vector<Result> out(64);
  for (double f : {60e6, 300e6}) fails += orc_trace_pixels(&m, &P, &im, f, 64, pix.data(), out.data(), 2);
  P.carried_tube = 1;
  fails += orc_trace_pixels(&m, &P, &im, 120e6, 64, pix.data(), out.data(), 2);
  P.carried_tube = 0;
  std::vector<double> path(size_t(4000) * 12);
  int plen = 0;
  fails += orc_trace_pixel_path(&m, &P, &im, 80e6, 27, out.data(), path.data(), 4000, &plen);
  // Dormand-Prince on an analytic medium, launched rays
  Medium ba{};
  ba.kind = ANALYTIC_BA; ba.r_in = 1.0; ba.r_max = 3.0; ba.t_const = 1e6;
  Params Q = P;
  Q.stepper = 1; Q.twin_check = 0;
  const double r0[6] = {2.9, 0.5, 0.2, 2.5, 1.2, -0.4};
  const double dir[6] = {-1, 0, 0, -1, 0.1, 0};
  std::vector<Result> two(2);
  fails += orc_trace_launch(&ba, &Q, 80e6, 2, r0, dir, two.data(), nullptr, 0, nullptr, 2);
  // Cartesian grid
  std::vector<float> cne(size_t(9) * 9 * 9), cte(cne.size(), 1e6f);
  for (size_t i = 0; i < cne.size(); ++i) cne[i] = float(1e6 + 1e4 * double(i % 9));
  Medium cm{};
  cm.kind = GRID_CARTESIAN; cm.n0 = cm.n1 = cm.n2 = 9;
  cm.r_in = -1.0; cm.r_max = 3.0;
  for (int k = 0; k < 3; ++k) { cm.origin[k] = -4.0; cm.spacing[k] = 1.0; }
  cm.ne = cne.data(); cm.te = cte.data();
  fails += orc_trace_pixels(&cm, &P, &im, 50e6, 64, pix.data(), out.data(), 2);
  // medium probe and free-free coefficient
  const double pos[6] = {1.5, 0.1, 0.2, 0.0, 0.0, 2.0};
  double ev[10];
  fails += orc_eval_medium(&m, 2, pos, ev);
  const double nes[2] = {1e8, 1e7}, tes[2] = {1e6, 1e5};
  double kn[2];
  fails += orc_kappa_n(2, nes, tes, 100e6, kn);
  // dual numbers and tapes on a 4 x 4 image at two frequencies
  Image small = im;
  small.nu = small.nv = 4; small.half_u = small.half_v = 2.0;
  const double freqs[2] = {90e6, 250e6};
  std::vector<float> w(32, 1.0f);
  w[5] = 0.0f;
  std::vector<double> vn(ne.size(), 0.01), vt(ne.size(), -0.02);
  double loss = 0, dl = 0;
  P.twin_check = 0;
  fails += orc_dual_loss(&m, &P, &small, 2, freqs, w.data(), vn.data(), vt.data(), &loss, &dl, 2);
  std::vector<double> gne(ne.size()), gte(ne.size());
  fails += orc_grad_loss(&m, &P, &small, 2, freqs, w.data(), &loss, gne.data(), gte.data(), 2);
  if (fails != 0 || !std::isfinite(loss) || !std::isfinite(dl) || plen < 1) {
    std::printf("failed: status sum %d, loss %g, dloss %g, path %d\n", fails, loss, dl, plen);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
