// Exercises every function of the oracle (oracle/lbm_oracle.h) on small
// lattices and on rejected arguments, for a build with the address and
// undefined-behaviour sanitizers (tests/test_oracle_sanitized.py).  Exits 0
// when every call returned what it should; the sanitizers abort on any
// out-of-bounds access, use of freed memory or undefined operation.
#include <cmath>
#include <cstdio>
#include <vector>

#include "lbm_oracle.h"

static int failures = 0;
#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::fprintf(stderr, "line %d: %s failed\n", __LINE__, #cond);  \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static orc_params params(int eq_kind, int source_on) {
  orc_params p{};
  p.lambda = eq_kind == 1 ? 1.0 : 1.3;
  p.rho0 = eq_kind == 1 ? 1.0 : 1.1;
  p.cp = eq_kind == 1 ? 1.0 : 1.7;
  p.gamma = 1.4;
  p.prandtl = 0.8;
  p.c0 = 0.5;
  p.s0 = 0.1;
  p.dx = 1.0;
  p.s_e = 1.6;
  p.s_psi = 1.4;
  p.s_eps = 1.5;
  p.u0_lin = 0.1;
  p.s0_lin = 0.2;
  p.alpha = 0.3;
  p.source_on = eq_kind >= 2 ? 0 : source_on;
  p.eq_kind = eq_kind;
  return p;
}

static void exercise(int64_t n, const orc_params& p) {
  std::vector<double> rho(n), J(n), zeta(n), d1(n), d2(n), d3(n), tgt(n);
  for (int64_t j = 0; j < n; ++j) {
    rho[j] = p.rho0 * (1.0 + 0.1 * std::sin(0.7 * j));
    J[j] = 0.05 * std::cos(0.3 * j);
    zeta[j] = rho[j] * (p.s0 + 0.1 * std::sin(1.1 * j));
    d1[j] = std::cos(0.5 * j);
    d2[j] = std::sin(0.9 * j);
    d3[j] = 0.1;
    tgt[j] = p.rho0;
  }
  const size_t S = 6 * (size_t)n;
  std::vector<double> f(S), g(S), m(S), df(S), dg(S), fb(S), fb2(S), eq(5 * n),
      dz(n), a(n), b(n), c(n);
  double M[36], Minv[36], diag[8], rbar[3] = {0, 0, 0}, dr[3] = {0.1, -0.2, 0.3};
  double L = 0, dL = 0;
  EXPECT(orc_moment_matrix(&p, M, Minv) == 0);
  EXPECT(orc_init(n, rho.data(), J.data(), zeta.data(), &p, f.data()) == 0);
  EXPECT(orc_moments(n, f.data(), &p, m.data()) == 0);
  EXPECT(orc_equilibria(n, rho.data(), J.data(), zeta.data(), &p, eq.data()) == 0);
  EXPECT(orc_source(n, f.data(), &p, dz.data()) == 0);
  EXPECT(orc_step(n, f.data(), &p, g.data()) == 0);
  EXPECT(orc_run(n, g.data(), 3, &p) == 0);
  EXPECT(orc_diagnostics(n, g.data(), &p, diag) == 0);
  EXPECT(diag[6] == 0 && diag[7] == 0);
  for (size_t i = 0; i < S; ++i) df[i] = std::sin(0.37 * i);
  EXPECT(orc_step_tlm(n, f.data(), df.data(), dr, &p, g.data(), dg.data()) == 0);
  EXPECT(orc_step_adjoint(n, f.data(), df.data(), &p, fb.data(), rbar) == 0);
  EXPECT(orc_init_tlm(n, rho.data(), J.data(), zeta.data(), d1.data(), d2.data(),
                      d3.data(), &p, g.data(), dg.data()) == 0);
  EXPECT(orc_init_adjoint(n, rho.data(), J.data(), zeta.data(), fb.data(), &p,
                          a.data(), b.data(), c.data()) == 0);
  EXPECT(orc_loss(n, f.data(), tgt.data(), &p, &L, fb2.data()) == 0);
  for (int64_t ck : {0, 1, 3, 7}) {
    EXPECT(orc_gradient(n, rho.data(), J.data(), zeta.data(), 7, ck, tgt.data(),
                        &p, &L, a.data(), b.data(), c.data(), rbar) == 0);
  }
  EXPECT(orc_gradient(n, rho.data(), J.data(), zeta.data(), 0, 0, tgt.data(), &p,
                      &L, a.data(), b.data(), c.data(), rbar) == 0);
  EXPECT(orc_directional(n, rho.data(), J.data(), zeta.data(), d1.data(),
                         d2.data(), d3.data(), dr, 5, tgt.data(), &p, &L,
                         &dL) == 0);
  // rejected arguments return -1 without touching memory
  EXPECT(orc_step(2, f.data(), &p, g.data()) == -1);
  EXPECT(orc_step(n, nullptr, &p, g.data()) == -1);
  EXPECT(orc_step(n, f.data(), &p, f.data()) == -1);
  EXPECT(orc_run(n, f.data(), -1, &p) == -1);
  EXPECT(orc_moments(n, f.data(), nullptr, m.data()) == -1);
  orc_params bad = p;
  bad.s_e = 2.0;
  EXPECT(orc_init(n, rho.data(), J.data(), zeta.data(), &bad, f.data()) == -1);
  bad = p;
  bad.gamma = 1.0;
  EXPECT(orc_diagnostics(n, f.data(), &bad, diag) == -1);
}

int main() {
  double s_psi = 0, s_eps = 0, s_e = 0;
  EXPECT(orc_coupled_rates(1.9, 1.4, 1.0, &s_psi, &s_eps) == 0);
  EXPECT(orc_coupled_rates(2.5, 1.4, 1.0, &s_psi, &s_eps) == -1);
  EXPECT(orc_rate_from_viscosity(6.579e-4, 1.0, 1.0 / 40, &s_e) == 0);
  EXPECT(orc_rate_from_viscosity(-1.0, 1.0, 1.0, &s_e) == -1);
  for (int kind = 0; kind <= 3; ++kind)
    for (int src = 0; src <= 1; ++src)
      for (int64_t n : {3, 4, 5, 17})
        exercise(n, params(kind, src));
  std::printf("oracle sanitizer driver: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
