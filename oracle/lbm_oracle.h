/*
 * Reference oracle for the coupled D1Q3Q3 lattice Boltzmann scheme of
 * Dubois, Graille & Lallemand, "Recovering the full Navier Stokes equations
 * with lattice Boltzmann schemes" (arXiv 1802.02369).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 CPU
 * implementation written from the paper.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Conventions
 *   - A lattice of n nodes is periodic.  A state is six FP64 arrays of
 *     length n laid end to end (SoA): f0, f+, f-, g0, g+, g- (the particle
 *     vector f_d of section 6).
 *   - Every function returns 0 on success and a negative value on bad
 *     arguments (null pointer, n < 3, non-positive constants, rates outside
 *     (0, 2)).  Nothing is allocated that outlives a call.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
  double lambda;   /* lattice velocity dx/dt (section 2) */
  double rho0;     /* scale factor of M and reference density of the EOS */
  double cp;       /* specific heat at constant pressure */
  double gamma;    /* cp / cv */
  double prandtl;  /* rho nu cp / kappa (section 5) */
  double c0;       /* reference sound speed, c0^2 = gamma p0 / rho0 */
  double s0;       /* reference specific entropy of the EOS */
  double dx;       /* space step; the scheme depends on it only through nu */
  double s_e, s_psi, s_eps; /* relaxation rates of e, psi, eps */
  double u0_lin, s0_lin;    /* reference state of the linearised equilibria;
                               u0_lin is also the advection velocity u0 of
                               the thermal scheme (eq_kind 3) */
  double alpha;             /* eps_eq = alpha lambda^2 zeta (eq_kind 3) */
  int32_t source_on;        /* 1: add the entropy-production source, step (vii) */
  int32_t eq_kind;          /* 0: nonlinear equilibria of section 8;
                               1: linear equilibria of section 7;
                               2: the fluid D1Q3 scheme of sections 2-3
                                  (isentropic pressure), g passive;
                               3: the thermal D1Q3 advection-diffusion
                                  scheme of section 4, f passive */
} orc_params;

/* Relaxation-rate coupling of section 7 (eq. lien-sigma-sigma) and the
   choice s_eps = 1.5 of step (iii). */
int orc_coupled_rates(double s_e, double gamma, double prandtl,
                      double* s_psi, double* s_eps);
/* Inverse of nu = sigma_e lambda dx (eq. nu-d1q3q3) with sigma = 1/s - 1/2. */
int orc_rate_from_viscosity(double nu, double lambda, double dx, double* s_e);

/* The 6x6 moment matrix M_D1Q3Q3 (row-major, moment order rho, J, zeta, e,
   psi, eps) and its numerical inverse. */
int orc_moment_matrix(const orc_params* p, double M[36], double Minv[36]);

/* m = M f_d at every node; m is SoA [6][n] in the order above. */
int orc_moments(int64_t n, const double* f, const orc_params* p, double* m);
/* Equilibria and thermodynamics from conserved moments:
   out is SoA [5][n]: e_eq, psi_eq, eps_eq, p, T. */
int orc_equilibria(int64_t n, const double* rho, const double* J,
                   const double* zeta, const orc_params* p, double* out);
/* Entropy source increment dt*S_j of step (vii) at every node, computed from
   the state f at time t. */
int orc_source(int64_t n, const double* f, const orc_params* p, double* dzeta);

/* Equilibrium initialisation f = M^-1 (rho, J, zeta, e_eq, psi_eq, eps_eq). */
int orc_init(int64_t n, const double* rho, const double* J, const double* zeta,
             const orc_params* p, double* f);
/* One time step (ii)-(viii): f_out = step(f_in).  f_out must not alias f_in. */
int orc_step(int64_t n, const double* f_in, const orc_params* p, double* f_out);
/* nsteps time steps in place. */
int orc_run(int64_t n, double* f, int64_t nsteps, const orc_params* p);

/* Diagnostics: out[0..7] = sum rho, sum J, sum zeta, sum rho E, min rho,
   min T, number of non-finite entries of f, number of nodes with rho<=0 or
   T<=0.  rho E = p/(gamma-1) + J^2/(2 rho) (section 5). */
int orc_diagnostics(int64_t n, const double* f, const orc_params* p,
                    double out[8]);

/* Tangent-linear step: (f_out, df_out) = (step(f), d step . (df, dr)) where
   dr = (d s_e, d s_psi, d s_eps).  Exact forward-mode derivative. */
int orc_step_tlm(int64_t n, const double* f, const double* df,
                 const double dr[3], const orc_params* p, double* f_out,
                 double* df_out);
/* Adjoint step: fbar = (d step/d f)^T fbar_next and
   rbar[q] += (d step/d rate_q)^T fbar_next, at the state f (time t). */
int orc_step_adjoint(int64_t n, const double* f, const double* fbar_next,
                     const orc_params* p, double* fbar, double rbar[3]);
/* Tangent and adjoint of the equilibrium initialisation in (rho, J, zeta). */
int orc_init_tlm(int64_t n, const double* rho, const double* J,
                 const double* zeta, const double* drho, const double* dJ,
                 const double* dzeta, const orc_params* p, double* f,
                 double* df);
int orc_init_adjoint(int64_t n, const double* rho, const double* J,
                     const double* zeta, const double* fbar,
                     const orc_params* p, double* rho_bar, double* J_bar,
                     double* zeta_bar);

/* Final-density misfit L = 1/2 sum_j (rho_j - target_j)^2 and its gradient
   with respect to the state f. */
int orc_loss(int64_t n, const double* f, const double* target,
             const orc_params* p, double* loss, double* fbar);

/* Gradient of L(rho(T)) for a run of nsteps from equilibrium initial data
   (rho, J, zeta): loss, d/d rho(0), d/d J(0), d/d zeta(0) and d/d rates.
   States are kept every ckpt steps and recomputed (ckpt <= 0: keep all). */
int orc_gradient(int64_t n, const double* rho, const double* J,
                 const double* zeta, int64_t nsteps, int64_t ckpt,
                 const double* target, const orc_params* p, double* loss,
                 double* rho_bar, double* J_bar, double* zeta_bar,
                 double rbar[3]);

/* Directional derivative of the same loss along (drho, dJ, dzeta, dr). */
int orc_directional(int64_t n, const double* rho, const double* J,
                    const double* zeta, const double* drho, const double* dJ,
                    const double* dzeta, const double dr[3], int64_t nsteps,
                    const double* target, const orc_params* p, double* loss,
                    double* dloss);

#ifdef __cplusplus
}
#endif
#endif
