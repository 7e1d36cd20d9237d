// sanitize_check.cpp -- drives the FP64 oracle through every mode on tiny
// channels, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
// (test infrastructure, like the oracle itself). Exits non-zero when a run
// gives a non-finite state; the sanitizers abort on their own findings.
//
//   g++ -std=c++17 -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all \
//       -fno-omit-frame-pointer oracle/wcsph_oracle.cpp oracle/sanitize_check.cpp
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "oracle.h"

namespace {

// A 24 x 16 mm channel at dx = 1 mm, disk of radius 3 mm at 300 m/s, the
// constants of the hot path.
orc_params tiny() {
  orc_params p;
  std::memset(&p, 0, sizeof p);
  p.L = 0.024; p.W = 0.016; p.dx = 1e-3; p.h_over_dx = 1.3; p.cell_size = 0.0;
  p.rho0 = 1000.0; p.c0 = 1480.0; p.gamma = 7.0; p.p_cav = -1e5;
  p.alpha = 0.1; p.delta = 0.1; p.eps_xsph = 0.02; p.mu_dyn = 8.9e-4; p.eta2 = 0.01;
  p.cfl = 0.2; p.gravity_y = -9.81;
  p.rho_lo = 0.5; p.rho_hi = 1.5; p.eps_wall = 1e-6;
  p.ghost_layers = 3; p.n_disk_ghosts = 100; p.ghost_rho_mode = 0; p.init_mode = 0;
  p.disk_R = 3e-3; p.disk_x0 = 3e-3; p.disk_y0 = 0.008; p.disk_mass = 8.01e-3;
  p.n_probes = 2;
  p.probe_xy[0] = 0.006; p.probe_xy[1] = 0.0;
  p.probe_xy[2] = 0.012; p.probe_xy[3] = 0.016;
  p.diag_every = 5;
  p.kin_mode = 0; p.kin_v0 = 300.0; p.kin_t_ramp = 5e-6; p.kin_coef = 1e5;
  p.mg_s1 = 1.979; p.mg_gamma0 = 0.11; p.mg_mu_max = 0.25; p.mg_a = 3.0;
  return p;
}

int failures = 0;

void run(const char* name, const orc_params& p, int steps, const std::vector<double>* kin_rows = nullptr) {
  void* s = orc_create(&p, 0, nullptr);
  if (!s) {
    std::printf("%s: not built\n", name);
    ++failures;
    return;
  }
  if (kin_rows) orc_set_kin_table(s, (int)(kin_rows->size() / 4), kin_rows->data());
  orc_step(s, steps);
  const int nf = orc_num_fluid(s), ng = orc_num_ghost(s);
  std::vector<double> a(nf), b(nf), c(nf), d(nf), e(nf), g1(ng), g2(ng), g3(ng), g4(ng);
  double t = 0.0, vmax = 0.0;
  orc_get_fluid(s, &t, a.data(), b.data(), c.data(), d.data(), e.data());
  bool ok = std::isfinite(t);
  for (int i = 0; i < nf; ++i) ok = ok && std::isfinite(a[i] + b[i] + c[i] + d[i] + e[i]);
  orc_eval_rates(s, a.data(), b.data(), c.data(), d.data(), e.data(), g1.data(), g2.data(), g3.data(),
                 g4.data(), &vmax);
  for (int i = 0; i < nf; ++i) ok = ok && std::isfinite(a[i] + b[i] + c[i] + d[i] + e[i]);
  const int rows = orc_probe_rows(s), nd = orc_diag_rows(s);
  std::vector<double> pt(rows), pdt(rows), pp((size_t)rows * p.n_probes), dg((size_t)nd * ORC_NDIAG);
  orc_get_probes(s, pt.data(), pdt.data(), pp.data());
  orc_get_diags(s, dg.data());
  for (double v : pp) ok = ok && std::isfinite(v);
  for (double v : dg) ok = ok && std::isfinite(v);
  std::vector<int> order(nf + ng), cs(orc_num_cells(s) + 1);
  orc_get_order(s, order.data(), cs.data());
  orc_destroy(s);
  std::printf("%s: %d fluid, %d steps, %s\n", name, nf, steps, ok ? "finite" : "NON-FINITE");
  if (!ok) ++failures;
}

}  // namespace

int main() {
  const orc_params base = tiny();
  run("wendland, predictor-corrector", base, 20);
  orc_params p = base;
  p.kernel_type = 1; p.alpha = 0.03; p.ghost_layers = 1;
  run("cubic spline, single-line walls", p, 20);
  p = base; p.eos_type = 1; p.c0 = 1448.0; p.ghost_rho_mode = 1;
  run("mie-grueneisen, eos inverse ghosts", p, 20);
  p = base; p.beta = 1.0; p.init_mode = 1;
  run("quadratic av, hydrostatic start", p, 20);
  p = base; p.kin_mode = 1; p.kin_coef = 0.383;
  run("quadratic drag", p, 20);
  p = base; p.kin_mode = 2;
  run("two-way coupled disk", p, 20);
  p = base; p.kin_mode = 3;
  const std::vector<double> rows = {0.0, 3e-3, 0.0, 6e7, 5e-6, 3.75e-3, 300.0, 0.0, 1e-4, 3.3e-2, 300.0, 0.0};
  run("tabulated disk motion", p, 20, &rows);
  p = base; p.scheme = 1; p.eos_type = 1; p.c0 = 1448.0; p.kernel_type = 1; p.cfl = 0.25; p.delta = 0.0;
  run("scheme 1 (summation density, leapfrog, internal energy)", p, 20);
  p = base; p.axisym = 1; p.W = 0.008; p.disk_y0 = 0.0; p.gravity_y = 0.0;
  p.probe_xy[3] = 0.008;
  run("axisymmetric r-z", p, 20);
  p = base; p.disk_R = 0.0; p.n_disk_ghosts = 0;
  run("no disk", p, 10);

  // building blocks
  std::vector<double> dt(5, 2e-8);
  double J = 0.0, dJ[3] = {0, 0, 0};
  orc_tangent_J(&base, 5, dt.data(), &J, dJ);
  if (!std::isfinite(J + dJ[0] + dJ[1] + dJ[2])) { std::printf("tangent: NON-FINITE\n"); ++failures; }
  const int n = 200;
  std::vector<double> x(n), y(n);
  for (int i = 0; i < n; ++i) {
    x[i] = 1e-3 * (0.37 * i - 25.0 * std::floor(0.37 * i / 25.0));
    y[i] = 1e-3 * (0.61 * i - 15.0 * std::floor(0.61 * i / 15.0));
  }
  std::vector<int> keys(n), perm(n), cst(4096), prs(2 * 20000);
  orc_cell_list(&base, n, x.data(), y.data(), keys.data(), perm.data(), cst.data());
  const long nb = orc_brute_pairs(&base, n, x.data(), y.data(), prs.data(), 20000);
  const long nc = orc_cell_pairs(&base, n, x.data(), y.data(), prs.data(), 20000);
  if (nb != nc) { std::printf("pairs: brute %ld cell %ld\n", nb, nc); ++failures; }
  double W, F, pr, c;
  orc_kernel_type(1, 0.5, 1.3e-3, &W, &F);
  orc_eos(&base, 1001.0, &pr, &c);
  orc_elastic_energy(&base, 900.0);
  orc_eos_rho(&base, 1e6);
  orc_lattice_mass(&base);
  std::printf("%s\n", failures ? "FAILED" : "sanitizer runs clean");
  return failures ? 1 : 0;
}
