// Reference oracle for the coupled D1Q3Q3 lattice Boltzmann scheme
// (Dubois, Graille & Lallemand, arXiv 1802.02369).
//
// TEST INFRASTRUCTURE ONLY: plain single-threaded FP64 loops that follow the
// paper's algorithm (section 8, steps (i)-(viii)) in its order and notation.
// Only the tests, the smoke check and the benchmark's CPU-baseline leg use
// it.  It shares no code with the GPU library.  Build without -ffast-math and
// with -ffp-contract=off.
//
// Readings of the paper taken here (each is listed with its reason in the
// design notes of the repository):
//   * eps_eq is taken in the polytropic form printed right after eq.
//     eq-energie-entropie-d1q3q3 (the paper's own specialisation to the EOS
//     of eq. gaz-parfait).  The general form with log(T/T0) agrees with it
//     exactly when T0 = T(rho0, s0), the temperature of the reference state;
//     p0 = rho0 c0^2 / gamma (section 7).
//   * Step (vii): the source dt*S_j, with S the right-hand side of the third
//     equation of eq. NS-rho-J-zeta, is added to zeta after the relaxation;
//     the equilibria use the pre-source zeta.  d_x u and d_x T are centred
//     differences of the time-t fields at j-1, j+1 (periodic).
//     nu = sigma_e lambda dx (eq. nu-d1q3q3), kappa = rho nu cp / Pr
//     (section 5), dt = dx / lambda (section 2).
//   * Gradients (tangent and adjoint) treat s_e, s_psi, s_eps as independent
//     inputs; s_e also enters the source through sigma_e.
#include "lbm_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Forward-mode dual numbers: value plus K partial derivatives.  Used to get
// exact derivatives of the very same step code (tangent-linear model) and the
// per-node Jacobian blocks from which the adjoint is assembled.
// ---------------------------------------------------------------------------
template <int K>
struct Dual {
  double v;
  double d[K];
};

template <int K>
Dual<K> dconst(double x) {
  Dual<K> r;
  r.v = x;
  for (int i = 0; i < K; ++i) r.d[i] = 0.0;
  return r;
}
template <int K>
Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v + b.v;
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int K>
Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v - b.v;
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int K>
Dual<K> operator-(const Dual<K>& a) {
  Dual<K> r;
  r.v = -a.v;
  for (int i = 0; i < K; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int K>
Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v * b.v;
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int K>
Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v / b.v;
  for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
template <int K>
Dual<K> operator+(const Dual<K>& a, double b) { return a + dconst<K>(b); }
template <int K>
Dual<K> operator+(double a, const Dual<K>& b) { return dconst<K>(a) + b; }
template <int K>
Dual<K> operator-(const Dual<K>& a, double b) { return a - dconst<K>(b); }
template <int K>
Dual<K> operator-(double a, const Dual<K>& b) { return dconst<K>(a) - b; }
template <int K>
Dual<K> operator*(const Dual<K>& a, double b) {
  Dual<K> r;
  r.v = a.v * b;
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int K>
Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K>
Dual<K> operator/(const Dual<K>& a, double b) { return a / dconst<K>(b); }
template <int K>
Dual<K> operator/(double a, const Dual<K>& b) { return dconst<K>(a) / b; }

template <int K>
Dual<K> exp(const Dual<K>& a) {
  Dual<K> r;
  r.v = std::exp(a.v);
  for (int i = 0; i < K; ++i) r.d[i] = r.v * a.d[i];
  return r;
}
template <int K>
Dual<K> log(const Dual<K>& a) {
  Dual<K> r;
  r.v = std::log(a.v);
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] / a.v;
  return r;
}
template <int K>
Dual<K> pow(const Dual<K>& a, double e) {
  Dual<K> r;
  r.v = std::pow(a.v, e);
  const double g = e * std::pow(a.v, e - 1.0);
  for (int i = 0; i < K; ++i) r.d[i] = g * a.d[i];
  return r;
}

inline double value(double x) { return x; }
template <int K>
double value(const Dual<K>& x) { return x.v; }

using std::exp;
using std::log;
using std::pow;

// ---------------------------------------------------------------------------
// Per-lattice context: the moment matrix, its inverse and derived constants.
// ---------------------------------------------------------------------------
struct Ctx {
  orc_params p;
  double M[6][6];
  double Minv[6][6];
  double r;   // gas constant cp (gamma - 1) / gamma, from c^2 = (gamma-1) cp T
  double p0;  // reference pressure rho0 c0^2 / gamma (section 7)
  double T0;  // reference temperature T(rho0, s0) = p0 / (rho0 r)
  double dt;  // dx / lambda
};

bool valid_rate(double s) { return s > 0.0 && s < 2.0 && std::isfinite(s); }

// Gauss-Jordan elimination with partial pivoting on a 6x6 matrix.
bool invert6(const double A[6][6], double B[6][6]) {
  double a[6][12];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 12; ++j)
      a[i][j] = j < 6 ? A[i][j] : (j - 6 == i ? 1.0 : 0.0);
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int i = c + 1; i < 6; ++i)
      if (std::fabs(a[i][c]) > std::fabs(a[piv][c])) piv = i;
    if (a[piv][c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 12; ++j) {
        double t = a[c][j];
        a[c][j] = a[piv][j];
        a[piv][j] = t;
      }
    const double d = a[c][c];
    for (int j = 0; j < 12; ++j) a[c][j] /= d;
    for (int i = 0; i < 6; ++i) {
      if (i == c) continue;
      const double fct = a[i][c];
      if (fct != 0.0)
        for (int j = 0; j < 12; ++j) a[i][j] -= fct * a[c][j];
    }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) B[i][j] = a[i][j + 6];
  return true;
}

// Builds the context; returns false on invalid parameters.
bool make_ctx(const orc_params* p, Ctx* c) {
  if (!p) return false;
  const double pos[] = {p->lambda, p->rho0, p->cp, p->prandtl, p->c0, p->dx};
  for (double v : pos)
    if (!(v > 0.0) || !std::isfinite(v)) return false;
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return false;
  if (!valid_rate(p->s_e) || !valid_rate(p->s_psi) || !valid_rate(p->s_eps))
    return false;
  if (p->eq_kind < 0 || p->eq_kind > 3) return false;
  // The linear equilibria of section 7 are printed in units lambda = cp = 1.
  if (p->eq_kind == 1 && (p->lambda != 1.0 || p->cp != 1.0 || p->rho0 != 1.0))
    return false;
  // The single-distribution schemes carry no temperature source; the
  // thermal one is stable for -2 < alpha < 1 (section 4).
  if (p->eq_kind >= 2 && p->source_on) return false;
  if (p->eq_kind == 3 && !(p->alpha > -2.0 && p->alpha < 1.0)) return false;
  c->p = *p;
  const double l = p->lambda, cp = p->cp, r0 = p->rho0;
  // Eq. M-d1q3q3: rows (rho, J, zeta, e, psi, eps), columns (f0, f+, f-,
  // g0, g+, g-).
  const double M[6][6] = {
      {1, 1, 1, 0, 0, 0},
      {0, l, -l, 0, 0, 0},
      {0, 0, 0, cp, cp, cp},
      {-2 * l * l, l * l, l * l, 0, 0, 0},
      {0, 0, 0, 0, cp * l, -cp * l},
      {0, 0, 0, -2 * cp * l * l, cp * l * l, cp * l * l},
  };
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) c->M[i][j] = r0 * M[i][j];
  if (!invert6(c->M, c->Minv)) return false;
  c->r = p->cp * (p->gamma - 1.0) / p->gamma;
  c->p0 = p->rho0 * p->c0 * p->c0 / p->gamma;
  c->T0 = c->p0 / (p->rho0 * c->r);
  c->dt = p->dx / p->lambda;
  return true;
}

// Thermodynamic state from conserved moments: u = J / rho, s = zeta / rho,
// p from eq. gaz-parfait, T from p = rho r T.
template <class S>
void thermo(const Ctx& c, const S& rho, const S& J, const S& zeta, S& u, S& s,
            S& pr, S& T) {
  const orc_params& p = c.p;
  u = J / rho;
  s = zeta / rho;
  pr = c.p0 * pow(rho / p.rho0, p.gamma) * exp(p.gamma * (s - p.s0) / p.cp);
  T = pr / (rho * c.r);
}

// Step (iv): equilibria of the non-conserved moments.
template <class S>
void equilibria(const Ctx& c, const S& rho, const S& J, const S& zeta,
                const S& u, const S& s, const S& pr, const S& T, S& e_eq,
                S& psi_eq, S& eps_eq) {
  const orc_params& p = c.p;
  const double l2 = p.lambda * p.lambda;
  if (p.eq_kind == 0) {
    // Eq. energie-equilibre, eq. psi-equilibre, and eq.
    // eq-energie-entropie-d1q3q3 in the form the paper gives it for the
    // polytropic gas of eq. gaz-parfait (the formula printed right after it):
    // eps_eq = 2 lambda^2 [rho (s - s0) + (1 - 1/gamma) cp rho log(rho/rho0)]
    //          + [3 (rho u^2 + p) - 2 lambda^2 rho] s.
    e_eq = 3.0 * (rho * u * u + pr) - 2.0 * l2 * rho;
    psi_eq = zeta * u;
    eps_eq = 2.0 * l2 *
                 (rho * (s - p.s0) +
                  (1.0 - 1.0 / p.gamma) * p.cp * rho * log(rho / p.rho0)) +
             (3.0 * (rho * u * u + pr) - 2.0 * l2 * rho) * s;
  } else if (p.eq_kind == 2) {
    // Section 2-3: fluid D1Q3 for the isentropic equations, eq.
    // energie-equilibre with the isentropic pressure p0 (rho/rho0)^gamma.
    // The entropy distribution is left passive (psi_eq = eps_eq = 0).
    const S p_iso = c.p0 * pow(rho / p.rho0, p.gamma);
    e_eq = 3.0 * (rho * u * u + p_iso) - 2.0 * l2 * rho;
    psi_eq = 0.0 * rho;
    eps_eq = 0.0 * rho;
  } else if (p.eq_kind == 3) {
    // Section 4: thermal D1Q3, psi_eq = u0 zeta, eps_eq = alpha lambda^2 zeta.
    // The fluid distribution is left passive with the linear acoustic
    // equilibrium e_eq = (3 c0^2 - 2 lambda^2) rho.
    e_eq = (3.0 * p.c0 * p.c0 - 2.0 * l2) * rho;
    psi_eq = p.u0_lin * zeta;
    eps_eq = p.alpha * l2 * zeta;
  } else {
    // Eq. equilibres-NS-linearise (units lambda = cp = 1), with the zeta
    // coefficient of e_eq read as 3 c0^2 / cp where the print shows
    // 3 u0^2 / cp: the first-order flux (2/3) lambda^2 rho + e_eq / 3 must be
    // the flux of J in eq. NS-rho-J-zeta-linearise, whose zeta term is
    // (c0^2 / cp) d_x zeta, and only with that term do the printed psi_eq
    // and eps_eq give the entropy equation of that system at second order
    // (eq. edp-ordre-2) for every u0, s0.
    const double u0 = p.u0_lin, s0 = p.s0_lin, c0 = p.c0, g = p.gamma;
    e_eq = (3.0 * (1.0 - s0 / p.cp) * c0 * c0 - 3.0 * u0 * u0 - 2.0 * l2) * rho +
           6.0 * u0 * J + 3.0 * (c0 * c0 / p.cp) * zeta;
    psi_eq = -u0 * s0 * rho + s0 * J + u0 * zeta;
    eps_eq = (-3.0 * (s0 * c0) * (s0 * c0) - 6.0 * s0 * u0 * u0 +
              3.0 * s0 * c0 * c0 + 2.0 - 2.0 * s0 - 2.0 / g) *
                 rho +
             6.0 * u0 * s0 * J + 3.0 * (p.cp * u0 * u0 + s0 * c0 * c0) * zeta;
  }
}

// u and T at a node from its six populations (used for the neighbours of
// step (vii)).
template <class S>
void node_uT(const Ctx& c, const S f[6], S& u, S& T) {
  S m[6];
  for (int i = 0; i < 6; ++i) {
    m[i] = c.M[i][0] * f[0];
    for (int k = 1; k < 6; ++k) m[i] = m[i] + c.M[i][k] * f[k];
  }
  S s, pr;
  thermo(c, m[0], m[1], m[2], u, s, pr, T);
}

// Step (vii): dt * S_j with S = rho nu / T (d_x u)^2 + kappa / T^2 (d_x T)^2,
// the right-hand side of the third equation of eq. NS-rho-J-zeta, using
// second-order centred differences of the time-t fields at j-1 and j+1,
// nu = sigma_e lambda dx (eq. nu-d1q3q3), kappa = rho nu cp / Pr (section 5).
template <class S>
S source_increment(const Ctx& c, const S& rho, const S& T, const S& uL,
                   const S& TL, const S& uR, const S& TR, const S& s_e) {
  const orc_params& p = c.p;
  const S sigma_e = 1.0 / s_e - 0.5;
  const S nu = sigma_e * p.lambda * p.dx;
  const S kappa = rho * nu * p.cp / p.prandtl;
  const S dxu = (uR - uL) / (2.0 * p.dx);
  const S dxT = (TR - TL) / (2.0 * p.dx);
  const S src = rho * nu / T * dxu * dxu + kappa / (T * T) * dxT * dxT;
  return c.dt * src;
}

// Steps (ii)-(vii) at one node: the post-collision populations f*, given the
// node's populations f, the time-t velocity and temperature of its left and
// right neighbours, and the three relaxation rates.
template <class S>
void collide_node(const Ctx& c, const S f[6], const S& uL, const S& TL,
                  const S& uR, const S& TR, const S rate[3], S fstar[6]) {
  const orc_params& p = c.p;
  // (ii) m = M f_d.
  S m[6];
  for (int i = 0; i < 6; ++i) {
    m[i] = c.M[i][0] * f[0];
    for (int k = 1; k < 6; ++k) m[i] = m[i] + c.M[i][k] * f[k];
  }
  const S rho = m[0], J = m[1], zeta = m[2], e = m[3], psi = m[4], eps = m[5];
  // (iii) rates are inputs; sigma_e (eq. henon-d1q3q3) feeds the viscosity.
  const S s_e = rate[0], s_psi = rate[1], s_eps = rate[2];
  // (iv) equilibria.
  S u, s, pr, T;
  thermo(c, rho, J, zeta, u, s, pr, T);
  S e_eq, psi_eq, eps_eq;
  equilibria(c, rho, J, zeta, u, s, pr, T, e_eq, psi_eq, eps_eq);
  // (v) relaxation, eq. relaxation-d1q3q3.
  const S e_s = e + s_e * (e_eq - e);
  const S psi_s = psi + s_psi * (psi_eq - psi);
  const S eps_s = eps + s_eps * (eps_eq - eps);
  // (vi) f_d* = M^-1 (rho, J, zeta, e*, psi*, eps*).
  const S ms[6] = {rho, J, zeta, e_s, psi_s, eps_s};
  for (int i = 0; i < 6; ++i) {
    fstar[i] = c.Minv[i][0] * ms[0];
    for (int k = 1; k < 6; ++k) fstar[i] = fstar[i] + c.Minv[i][k] * ms[k];
  }
  // (vii) dt * S_j is added to the conserved moment zeta, i.e.
  // M^-1 (0, 0, dt S_j, 0, 0, 0) is added to f_d*.
  if (p.source_on) {
    const S dz = source_increment(c, rho, T, uL, TL, uR, TR, s_e);
    for (int i = 0; i < 6; ++i) fstar[i] = fstar[i] + c.Minv[i][2] * dz;
  }
}

inline int64_t wrap(int64_t j, int64_t n) { return ((j % n) + n) % n; }

// (viii) eq. iteration-d1q3q3: f0, g0 stay; f+, g+ come from the left
// neighbour; f-, g- from the right neighbour.
template <class S>
void stream(int64_t n, const std::vector<S>& fs, S* out) {
  for (int64_t j = 0; j < n; ++j) {
    const int64_t jl = wrap(j - 1, n), jr = wrap(j + 1, n);
    for (int b = 0; b < 2; ++b) {
      out[(3 * b + 0) * n + j] = fs[(3 * b + 0) * n + j];
      out[(3 * b + 1) * n + j] = fs[(3 * b + 1) * n + jl];
      out[(3 * b + 2) * n + j] = fs[(3 * b + 2) * n + jr];
    }
  }
}

// One full time step on a periodic lattice, for any scalar type.
template <class S>
void step_generic(const Ctx& c, int64_t n, const S* f, const S rate[3],
                  S* out) {
  std::vector<S> u(n), T(n), fs(6 * n);
  for (int64_t j = 0; j < n; ++j) {
    S fj[6];
    for (int k = 0; k < 6; ++k) fj[k] = f[k * n + j];
    node_uT(c, fj, u[j], T[j]);
  }
  for (int64_t j = 0; j < n; ++j) {
    S fj[6], st[6];
    for (int k = 0; k < 6; ++k) fj[k] = f[k * n + j];
    const int64_t jl = wrap(j - 1, n), jr = wrap(j + 1, n);
    collide_node(c, fj, u[jl], T[jl], u[jr], T[jr], rate, st);
    for (int k = 0; k < 6; ++k) fs[k * n + j] = st[k];
  }
  stream(n, fs, out);
}

// Equilibrium populations at one node.
template <class S>
void init_node(const Ctx& c, const S& rho, const S& J, const S& zeta,
               S f[6]) {
  S u, s, pr, T, e_eq, psi_eq, eps_eq;
  thermo(c, rho, J, zeta, u, s, pr, T);
  equilibria(c, rho, J, zeta, u, s, pr, T, e_eq, psi_eq, eps_eq);
  const S m[6] = {rho, J, zeta, e_eq, psi_eq, eps_eq};
  for (int i = 0; i < 6; ++i) {
    f[i] = c.Minv[i][0] * m[0];
    for (int k = 1; k < 6; ++k) f[i] = f[i] + c.Minv[i][k] * m[k];
  }
}

// Adjoint of one step, assembled from exact per-node Jacobian blocks.
// f*(j) depends on f(j-1), f(j), f(j+1) (18 inputs) and the three rates.
using D21 = Dual<21>;

void step_adjoint(const Ctx& c, int64_t n, const double* f,
                  const double* fbar_next, double* fbar, double rbar[3]) {
  for (int64_t i = 0; i < 6 * n; ++i) fbar[i] = 0.0;
  const double rates[3] = {c.p.s_e, c.p.s_psi, c.p.s_eps};
  for (int64_t j = 0; j < n; ++j) {
    const int64_t nb[3] = {wrap(j - 1, n), j, wrap(j + 1, n)};
    D21 fin[3][6];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 6; ++k) {
        fin[a][k] = dconst<21>(f[k * n + nb[a]]);
        fin[a][k].d[6 * a + k] = 1.0;
      }
    D21 rate[3];
    for (int q = 0; q < 3; ++q) {
      rate[q] = dconst<21>(rates[q]);
      rate[q].d[18 + q] = 1.0;
    }
    D21 uL, TL, uR, TR, st[6];
    node_uT(c, fin[0], uL, TL);
    node_uT(c, fin[2], uR, TR);
    collide_node(c, fin[1], uL, TL, uR, TR, rate, st);
    // Adjoint of the streaming: f*(j) of population k went to node
    // j, j+1 or j-1 at time t+1.
    double sbar[6];
    for (int b = 0; b < 2; ++b) {
      sbar[3 * b + 0] = fbar_next[(3 * b + 0) * n + j];
      sbar[3 * b + 1] = fbar_next[(3 * b + 1) * n + wrap(j + 1, n)];
      sbar[3 * b + 2] = fbar_next[(3 * b + 2) * n + wrap(j - 1, n)];
    }
    for (int r = 0; r < 6; ++r) {
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 6; ++k)
          fbar[k * n + nb[a]] += st[r].d[6 * a + k] * sbar[r];
      for (int q = 0; q < 3; ++q) rbar[q] += st[r].d[18 + q] * sbar[r];
    }
  }
}

bool bad(int64_t n, const void* a) { return n < 3 || a == nullptr; }

}  // namespace

extern "C" {

int orc_coupled_rates(double s_e, double gamma, double prandtl, double* s_psi,
                      double* s_eps) {
  if (!valid_rate(s_e) || !(gamma > 1.0) || !(prandtl > 0.0) || !s_psi ||
      !s_eps)
    return -1;
  const double sigma_e = 1.0 / s_e - 0.5;                  // eq. henon
  const double sigma_psi = 1.5 * gamma / prandtl * sigma_e;  // eq. lien-sigma-sigma
  *s_psi = 1.0 / (sigma_psi + 0.5);
  *s_eps = 1.5;  // step (iii)
  return 0;
}

int orc_rate_from_viscosity(double nu, double lambda, double dx, double* s_e) {
  if (!(nu > 0.0) || !(lambda > 0.0) || !(dx > 0.0) || !s_e) return -1;
  const double sigma_e = nu / (lambda * dx);  // eq. nu-d1q3q3
  *s_e = 1.0 / (sigma_e + 0.5);
  return 0;
}

int orc_moment_matrix(const orc_params* p, double M[36], double Minv[36]) {
  Ctx c;
  if (!M || !Minv || !make_ctx(p, &c)) return -1;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      M[6 * i + j] = c.M[i][j];
      Minv[6 * i + j] = c.Minv[i][j];
    }
  return 0;
}

int orc_moments(int64_t n, const double* f, const orc_params* p, double* m) {
  Ctx c;
  if (bad(n, f) || !m || !make_ctx(p, &c)) return -1;
  for (int64_t j = 0; j < n; ++j)
    for (int i = 0; i < 6; ++i) {
      double acc = c.M[i][0] * f[j];
      for (int k = 1; k < 6; ++k) acc = acc + c.M[i][k] * f[k * n + j];
      m[i * n + j] = acc;
    }
  return 0;
}

int orc_equilibria(int64_t n, const double* rho, const double* J,
                   const double* zeta, const orc_params* p, double* out) {
  Ctx c;
  if (n < 1 || !rho || !J || !zeta || !out || !make_ctx(p, &c)) return -1;
  for (int64_t j = 0; j < n; ++j) {
    double u, s, pr, T, e_eq, psi_eq, eps_eq;
    thermo(c, rho[j], J[j], zeta[j], u, s, pr, T);
    equilibria(c, rho[j], J[j], zeta[j], u, s, pr, T, e_eq, psi_eq, eps_eq);
    out[0 * n + j] = e_eq;
    out[1 * n + j] = psi_eq;
    out[2 * n + j] = eps_eq;
    out[3 * n + j] = pr;
    out[4 * n + j] = T;
  }
  return 0;
}

int orc_source(int64_t n, const double* f, const orc_params* p,
               double* dzeta) {
  Ctx c;
  if (bad(n, f) || !dzeta || !make_ctx(p, &c)) return -1;
  std::vector<double> u(n), T(n), rho(n);
  for (int64_t j = 0; j < n; ++j) {
    double fj[6];
    for (int k = 0; k < 6; ++k) fj[k] = f[k * n + j];
    node_uT(c, fj, u[j], T[j]);
    double r = c.M[0][0] * fj[0];
    for (int k = 1; k < 6; ++k) r = r + c.M[0][k] * fj[k];
    rho[j] = r;
  }
  for (int64_t j = 0; j < n; ++j) {
    const int64_t jl = wrap(j - 1, n), jr = wrap(j + 1, n);
    dzeta[j] = source_increment(c, rho[j], T[j], u[jl], T[jl], u[jr], T[jr],
                                p->s_e);
  }
  return 0;
}

int orc_init(int64_t n, const double* rho, const double* J, const double* zeta,
             const orc_params* p, double* f) {
  Ctx c;
  if (bad(n, rho) || !J || !zeta || !f || !make_ctx(p, &c)) return -1;
  for (int64_t j = 0; j < n; ++j) {
    double fj[6];
    init_node(c, rho[j], J[j], zeta[j], fj);
    for (int k = 0; k < 6; ++k) f[k * n + j] = fj[k];
  }
  return 0;
}

int orc_step(int64_t n, const double* f_in, const orc_params* p,
             double* f_out) {
  Ctx c;
  if (bad(n, f_in) || !f_out || f_out == f_in || !make_ctx(p, &c)) return -1;
  const double rate[3] = {p->s_e, p->s_psi, p->s_eps};
  step_generic(c, n, f_in, rate, f_out);
  return 0;
}

int orc_run(int64_t n, double* f, int64_t nsteps, const orc_params* p) {
  Ctx c;
  if (bad(n, f) || nsteps < 0 || !make_ctx(p, &c)) return -1;
  const double rate[3] = {p->s_e, p->s_psi, p->s_eps};
  std::vector<double> tmp(6 * n);
  for (int64_t t = 0; t < nsteps; ++t) {
    step_generic(c, n, f, rate, tmp.data());
    std::memcpy(f, tmp.data(), sizeof(double) * 6 * n);
  }
  return 0;
}

int orc_diagnostics(int64_t n, const double* f, const orc_params* p,
                    double out[8]) {
  Ctx c;
  if (bad(n, f) || !out || !make_ctx(p, &c)) return -1;
  double srho = 0, sJ = 0, sz = 0, sE = 0, mrho = INFINITY, mT = INFINITY;
  double nonfinite = 0, nonphys = 0;
  for (int64_t j = 0; j < n; ++j) {
    double m[6];
    for (int i = 0; i < 6; ++i) {
      if (!std::isfinite(f[i * n + j])) nonfinite += 1;
      double acc = c.M[i][0] * f[j];
      for (int k = 1; k < 6; ++k) acc = acc + c.M[i][k] * f[k * n + j];
      m[i] = acc;
    }
    double u, s, pr, T;
    thermo(c, m[0], m[1], m[2], u, s, pr, T);
    srho += m[0];
    sJ += m[1];
    sz += m[2];
    sE += pr / (p->gamma - 1.0) + m[1] * m[1] / (2.0 * m[0]);
    if (m[0] < mrho) mrho = m[0];
    if (T < mT) mT = T;
    if (!(m[0] > 0.0) || !(T > 0.0)) nonphys += 1;
  }
  out[0] = srho;
  out[1] = sJ;
  out[2] = sz;
  out[3] = sE;
  out[4] = mrho;
  out[5] = mT;
  out[6] = nonfinite;
  out[7] = nonphys;
  return 0;
}

int orc_step_tlm(int64_t n, const double* f, const double* df,
                 const double dr[3], const orc_params* p, double* f_out,
                 double* df_out) {
  Ctx c;
  if (bad(n, f) || !df || !dr || !f_out || !df_out || !make_ctx(p, &c))
    return -1;
  using D1 = Dual<1>;
  std::vector<D1> a(6 * n), b(6 * n);
  for (int64_t i = 0; i < 6 * n; ++i) {
    a[i].v = f[i];
    a[i].d[0] = df[i];
  }
  const double rates[3] = {p->s_e, p->s_psi, p->s_eps};
  D1 rate[3];
  for (int q = 0; q < 3; ++q) {
    rate[q].v = rates[q];
    rate[q].d[0] = dr[q];
  }
  step_generic(c, n, a.data(), rate, b.data());
  for (int64_t i = 0; i < 6 * n; ++i) {
    f_out[i] = b[i].v;
    df_out[i] = b[i].d[0];
  }
  return 0;
}

int orc_step_adjoint(int64_t n, const double* f, const double* fbar_next,
                     const orc_params* p, double* fbar, double rbar[3]) {
  Ctx c;
  if (bad(n, f) || !fbar_next || !fbar || !rbar || !make_ctx(p, &c))
    return -1;
  step_adjoint(c, n, f, fbar_next, fbar, rbar);
  return 0;
}

int orc_init_tlm(int64_t n, const double* rho, const double* J,
                 const double* zeta, const double* drho, const double* dJ,
                 const double* dzeta, const orc_params* p, double* f,
                 double* df) {
  Ctx c;
  if (bad(n, rho) || !J || !zeta || !drho || !dJ || !dzeta || !f || !df ||
      !make_ctx(p, &c))
    return -1;
  using D1 = Dual<1>;
  for (int64_t j = 0; j < n; ++j) {
    D1 r, q, z, fj[6];
    r.v = rho[j];
    r.d[0] = drho[j];
    q.v = J[j];
    q.d[0] = dJ[j];
    z.v = zeta[j];
    z.d[0] = dzeta[j];
    init_node(c, r, q, z, fj);
    for (int k = 0; k < 6; ++k) {
      f[k * n + j] = fj[k].v;
      df[k * n + j] = fj[k].d[0];
    }
  }
  return 0;
}

int orc_init_adjoint(int64_t n, const double* rho, const double* J,
                     const double* zeta, const double* fbar,
                     const orc_params* p, double* rho_bar, double* J_bar,
                     double* zeta_bar) {
  Ctx c;
  if (bad(n, rho) || !J || !zeta || !fbar || !rho_bar || !J_bar || !zeta_bar ||
      !make_ctx(p, &c))
    return -1;
  using D3 = Dual<3>;
  for (int64_t j = 0; j < n; ++j) {
    D3 r = dconst<3>(rho[j]), q = dconst<3>(J[j]), z = dconst<3>(zeta[j]);
    r.d[0] = 1.0;
    q.d[1] = 1.0;
    z.d[2] = 1.0;
    D3 fj[6];
    init_node(c, r, q, z, fj);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 6; ++k)
      for (int a = 0; a < 3; ++a) acc[a] += fj[k].d[a] * fbar[k * n + j];
    rho_bar[j] = acc[0];
    J_bar[j] = acc[1];
    zeta_bar[j] = acc[2];
  }
  return 0;
}

int orc_loss(int64_t n, const double* f, const double* target,
             const orc_params* p, double* loss, double* fbar) {
  Ctx c;
  if (bad(n, f) || !target || !loss || !fbar || !make_ctx(p, &c)) return -1;
  double L = 0.0;
  for (int64_t i = 0; i < 6 * n; ++i) fbar[i] = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double rho = c.M[0][0] * f[j];
    for (int k = 1; k < 6; ++k) rho = rho + c.M[0][k] * f[k * n + j];
    const double d = rho - target[j];
    L += 0.5 * d * d;
    for (int k = 0; k < 6; ++k) fbar[k * n + j] = c.M[0][k] * d;
  }
  *loss = L;
  return 0;
}

int orc_gradient(int64_t n, const double* rho, const double* J,
                 const double* zeta, int64_t nsteps, int64_t ckpt,
                 const double* target, const orc_params* p, double* loss,
                 double* rho_bar, double* J_bar, double* zeta_bar,
                 double rbar[3]) {
  Ctx c;
  if (bad(n, rho) || !J || !zeta || !target || !loss || !rho_bar || !J_bar ||
      !zeta_bar || !rbar || nsteps < 0 || !make_ctx(p, &c))
    return -1;
  if (ckpt <= 0 || ckpt > nsteps) ckpt = nsteps > 0 ? nsteps : 1;
  const double rate[3] = {p->s_e, p->s_psi, p->s_eps};
  const int64_t S = 6 * n;
  // Forward pass keeping the state at every multiple of ckpt.
  const int64_t nck = nsteps / ckpt + 1;
  std::vector<double> ck(nck * S), cur(S), nxt(S);
  orc_init(n, rho, J, zeta, p, cur.data());
  for (int64_t t = 0; t < nsteps; ++t) {
    if (t % ckpt == 0) std::memcpy(&ck[(t / ckpt) * S], cur.data(), 8 * S);
    step_generic(c, n, cur.data(), rate, nxt.data());
    cur.swap(nxt);
  }
  std::vector<double> fbar(S), fbar2(S);
  orc_loss(n, cur.data(), target, p, loss, fbar.data());
  rbar[0] = rbar[1] = rbar[2] = 0.0;
  // Reverse sweep, one checkpoint segment at a time.
  std::vector<double> seg;
  for (int64_t t0 = ((nsteps - 1) / ckpt) * ckpt; nsteps > 0 && t0 >= 0;
       t0 -= ckpt) {
    const int64_t len = std::min(ckpt, nsteps - t0);
    seg.assign(len * S, 0.0);
    std::memcpy(seg.data(), &ck[(t0 / ckpt) * S], 8 * S);
    for (int64_t k = 1; k < len; ++k)
      step_generic(c, n, &seg[(k - 1) * S], rate, &seg[k * S]);
    for (int64_t k = len - 1; k >= 0; --k) {
      step_adjoint(c, n, &seg[k * S], fbar.data(), fbar2.data(), rbar);
      fbar.swap(fbar2);
    }
  }
  return orc_init_adjoint(n, rho, J, zeta, fbar.data(), p, rho_bar, J_bar,
                          zeta_bar);
}

int orc_directional(int64_t n, const double* rho, const double* J,
                    const double* zeta, const double* drho, const double* dJ,
                    const double* dzeta, const double dr[3], int64_t nsteps,
                    const double* target, const orc_params* p, double* loss,
                    double* dloss) {
  Ctx c;
  if (bad(n, rho) || !J || !zeta || !drho || !dJ || !dzeta || !dr ||
      !target || !loss || !dloss || nsteps < 0 || !make_ctx(p, &c))
    return -1;
  using D1 = Dual<1>;
  const int64_t S = 6 * n;
  std::vector<double> f(S), df(S);
  orc_init_tlm(n, rho, J, zeta, drho, dJ, dzeta, p, f.data(), df.data());
  std::vector<D1> a(S), b(S);
  for (int64_t i = 0; i < S; ++i) {
    a[i].v = f[i];
    a[i].d[0] = df[i];
  }
  const double rates[3] = {p->s_e, p->s_psi, p->s_eps};
  D1 rate[3];
  for (int q = 0; q < 3; ++q) {
    rate[q].v = rates[q];
    rate[q].d[0] = dr[q];
  }
  for (int64_t t = 0; t < nsteps; ++t) {
    step_generic(c, n, a.data(), rate, b.data());
    a.swap(b);
  }
  double L = 0.0, dL = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    D1 r = c.M[0][0] * a[j];
    for (int k = 1; k < 6; ++k) r = r + c.M[0][k] * a[k * n + j];
    const double d = r.v - target[j];
    L += 0.5 * d * d;
    dL += d * r.d[0];
  }
  *loss = L;
  *dloss = dL;
  return 0;
}

}  // extern "C"
