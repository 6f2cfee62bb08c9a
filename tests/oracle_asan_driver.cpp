// Drives every entry point of the FP64 reference on small random cases (2D
// and 3D Cartesian, spherical, quasi-spherical), for a build under the
// address and undefined-behaviour sanitizers (tests/test_sanitizers.py).
// Prints "ok" when every call returned success.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../oracle/oracle.h"

namespace {

int fail(const char *what, int geom) {
  std::printf("FAIL %s (geom %d)\n", what, geom);
  return 1;
}

int run_case(int geom, int dim, std::mt19937_64 &rng) {
  orc_grid g{};
  g.geom = geom;
  g.dim = dim;
  g.n[0] = 12;
  g.n[1] = 10;
  g.n[2] = dim == 3 ? 8 : 1;
  if (geom == 0) {
    for (int a = 0; a < 3; ++a) {
      g.lo[a] = 0.0;
      g.hi[a] = g.n[a];
      g.periodic[a] = 1;
    }
  } else {
    g.lo[0] = 1.0;
    g.hi[0] = 6.0;
    g.lo[1] = 0.0;
    g.hi[1] = M_PI;
    g.lo[2] = 0.0;
    g.hi[2] = 1.0;
    g.vartheta = geom == 2 ? 0.3 : 0.0;
  }
  g.rho0 = 1.0;
  const int64_t np = orc_field_points(&g);
  std::uniform_real_distribution<double> U(-0.1, 0.1), O(0.0, 0.999), P(0.0, 6.28);
  std::vector<double> EB(6 * np), EB2(6 * np), J(3 * np), lamJ(3 * np), dEB(6 * np), vEB(6 * np);
  for (auto &x : EB) x = U(rng);
  for (auto &x : lamJ) x = U(rng);
  for (auto &x : vEB) x = U(rng);
  const int64_t n = 300;
  std::vector<int32_t> cell(3 * n), alive(n, 1), cprev(3 * n), perm(n);
  std::vector<double> offs(3 * n), u(3 * n), w(n, 1.0), phi(n), oprev(3 * n);
  for (int64_t p = 0; p < n; ++p) {
    for (int a = 0; a < 3; ++a) {
      cell[3 * p + a] = a < dim ? (int32_t)(rng() % g.n[a]) : 0;
      offs[3 * p + a] = a < dim ? O(rng) : 0.0;
      u[3 * p + a] = 5 * U(rng);
    }
    phi[p] = P(rng);
  }
  orc_species sp{};
  sp.n = n;
  sp.cell = cell.data();
  sp.offs = offs.data();
  sp.u = u.data();
  sp.w = w.data();
  sp.phi = geom == 0 ? nullptr : phi.data();
  sp.alive = alive.data();
  sp.cell_prev = cprev.data();
  sp.offs_prev = oprev.data();
  sp.perm = perm.data();
  const double q = -1.0, m = 1.0, dt = orc_dt_from_cfl(&g, 0.45);
  // adjoint and tangent first (they read the initial state)
  std::vector<double> du0(3 * n), dd0(3 * n), vu(3 * n), vd(3 * n), lu(3 * n);
  for (auto &x : vu) x = U(rng);
  for (auto &x : vd) x = U(rng);
  for (auto &x : lu) x = U(rng);
  double *dup = du0.data(), *ddp = dd0.data();
  const double *vup = vu.data(), *vdp = vd.data(), *lup = lu.data();
  double loss = 0.0, dloss = 0.0;
  if (orc_adjoint(&g, dt, 3, EB.data(), 1, &q, &m, &sp, lamJ.data(), &lup, nullptr, dEB.data(),
                  &dup, &ddp, &loss))
    return fail("adjoint", geom);
  if (orc_jvp(&g, dt, 3, EB.data(), vEB.data(), 1, &q, &m, &sp, &vup, &vdp, lamJ.data(), &lup,
              nullptr, &loss, &dloss))
    return fail("jvp", geom);
  const int32_t pusher[1] = {geom == 0 ? 3 : 1};
  const double eovr[1] = {0.9}, lmax[1] = {0.5};
  if (orc_run_pushers(&g, dt, 4, 2, 0, EB.data(), 1, &q, &m, pusher, eovr, lmax, &sp, J.data()))
    return fail("run_pushers", geom);
  if (orc_run(&g, dt, 4, 2, 4, EB.data(), 1, &q, &m, &sp, J.data())) return fail("run", geom);
  EB2 = EB;
  if (orc_faraday(&g, EB2.data(), 0.5 * dt)) return fail("faraday", geom);
  if (orc_ampere(&g, EB2.data(), J.data(), dt, 4 * M_PI)) return fail("ampere", geom);
  if (orc_filter(&g, J.data(), 2)) return fail("filter", geom);
  std::vector<int32_t> keys(n);
  if (orc_sort_keys(&g, n, cell.data(), alive.data(), keys.data())) return fail("sort_keys", geom);
  orc_sort_perm(n, keys.data(), perm.data());
  std::vector<double> out6(6 * n), E3(3 * n), B3(3 * n);
  orc_interp(&g, EB.data(), n, cell.data(), offs.data(), out6.data());
  orc_to_cart(&g, n, cell.data(), offs.data(), geom == 0 ? nullptr : phi.data(), out6.data(),
              E3.data(), B3.data());
  orc_boris(n, 0.1, E3.data(), B3.data(), u.data());
  orc_vay(n, 0.1, E3.data(), B3.data(), u.data());
  orc_gca(n, 0.1, E3.data(), B3.data(), u.data());
  if (geom != 0) {
    double x[3] = {3.5, 4.25, 0.0}, X[3], h[3], xb[3], ph = 0.0;
    orc_sqrt_h(&g, x, h);
    orc_code_to_cart(&g, x, 1.0, X);
    orc_cart_to_code(&g, X, xb, &ph);
    (void)orc_theta_of_T(&g, 1.0);
    (void)orc_T_of_theta(&g, 1.0);
    (void)orc_polar_area(&g, 3.5);
  }
  return 0;
}

}  // namespace

int main() {
  std::mt19937_64 rng(2511);
  const int cases[4][2] = {{0, 2}, {0, 3}, {1, 2}, {2, 2}};
  for (const auto &c : cases)
    if (run_case(c[0], c[1], rng)) return 1;
  std::printf("ok\n");
  return 0;
}
