/*
 * lbm.h - C ABI of the MI355X (gfx950) implementation of the coupled D1Q3Q3
 * lattice Boltzmann scheme of Dubois, Graille & Lallemand, "Recovering the
 * full Navier Stokes equations with lattice Boltzmann schemes"
 * (arXiv 1802.02369): one D1Q3 distribution f for mass and momentum, one D1Q3
 * distribution g for the volumic entropy zeta = rho s, with the entropy
 * production source term of the Navier-Stokes equations written in
 * (rho, J, zeta) form (section 6, eq. NS-rho-J-zeta).
 *
 * Conventions shared by every entry point
 *   - All floating point data are FP64.
 *   - A state of a lattice of n nodes is six device arrays of n doubles laid
 *     end to end (structure of arrays, 6*n doubles): f0, f+, f-, g0, g+, g-,
 *     the particle vector f_d of section 6.  Node j holds f_k[j] at
 *     state[k*n + j].  Lattices are periodic.
 *   - Pointers named "device" are device memory owned by the caller (for
 *     example torch tensors).  The library never allocates device memory:
 *     every call that needs scratch space takes a caller workspace whose
 *     size a *_workspace_bytes call reports.
 *   - "stream" is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     on it and return without waiting, except those documented as
 *     synchronising (they return host values).
 *   - Every int-returning call returns LBM_OK (0) or a negative LBM_E* code;
 *     lbm_last_error() then gives a message (thread-local).  On an error
 *     nothing has been enqueued unless the code is LBM_EHIP.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad pointer, size, constant or rate */
  LBM_EHIP = -2,       /* a HIP runtime call failed */
  LBM_EWORKSPACE = -3, /* workspace too small */
  LBM_ENONFINITE = -4, /* state holds NaN/Inf, rho <= 0 or T <= 0 */
  LBM_ENOTSUP = -5     /* option not supported by this build */
};

/* Per-lattice constants.
 *   lambda  lattice velocity dx/dt (section 2)
 *   rho0    scale factor of the moment matrix (eq. M-d1q3q3) and reference
 *           density of the equation of state (eq. gaz-parfait); must agree
 *   cp      specific heat at constant pressure; gamma = cp/cv > 1
 *   prandtl Pr = rho nu cp / kappa (section 5)
 *   c0      reference sound speed, p0 = rho0 c0^2 / gamma (section 7)
 *   s0      reference specific entropy of the equation of state
 *   s_e, s_psi, s_eps  relaxation rates of e, psi, eps, each in (0, 2)
 *           (eq. relaxation-d1q3q3); lbm_coupled_rates gives the coupling
 *           of section 7.  s_e also sets the viscosity of the source term,
 *           nu = (1/s_e - 1/2) lambda dx (eqs. henon-d1q3q3, nu-d1q3q3).
 *   u0_lin, s0_lin  reference state of the linearised equilibria
 *           (eq_kind = 1)
 *   source_on  1: add the entropy production of step (vii) of section 8
 *   eq_kind    0: nonlinear equilibria of section 8 (eqs. energie-equilibre,
 *              psi-equilibre, eq-energie-entropie-d1q3q3);
 *              1: linear equilibria of section 7 (eq. equilibres-NS-linearise,
 *              printed for lambda = cp = rho0 = 1; other values are rejected)
 */
typedef struct lbm_params {
  double lambda, rho0, cp, gamma, prandtl, c0, s0;
  double s_e, s_psi, s_eps;
  double u0_lin, s0_lin;
  int32_t source_on;
  int32_t eq_kind;
} lbm_params;

typedef struct lbm_handle lbm_handle;
typedef struct lbm_batch lbm_batch;

/* Kernel choice for lbm_step / lbm_batch_run. */
enum {
  LBM_KERNEL_AUTO = 0,    /* tuned choice (default) */
  LBM_KERNEL_PLAIN = 1,   /* one launch per time step, one node per thread */
  LBM_KERNEL_BLOCKED = 2  /* register-resident tiles, k steps per launch */
};

typedef struct lbm_tuning {
  int32_t kernel;          /* LBM_KERNEL_* */
  int32_t nodes_per_lane;  /* P: contiguous nodes per lane (blocked kernel) */
  int32_t steps_per_launch;/* K: time steps per launch (blocked kernel) */
  int32_t waves_per_group; /* wavefronts per workgroup (blocked kernel) */
} lbm_tuning;

/* ----------------------------------------------------------------- misc */

/* Message of the last failing call on this thread ("" if none). */
const char* lbm_last_error(void);

/* Relaxation coupling of section 7: sigma = 1/s - 1/2 (eq. henon),
 * sigma_psi = (3/2)(gamma/Pr) sigma_e (eq. lien-sigma-sigma), s_eps = 1.5
 * (step (iii) of section 8).  ds_psi_ds_e (may be NULL) receives the
 * derivative of s_psi with respect to s_e.  Host only. */
int lbm_coupled_rates(double s_e, double gamma, double prandtl, double* s_psi,
                      double* s_eps, double* ds_psi_ds_e);

/* ----------------------------------------------------- single lattice */

/* Creates a handle for one periodic lattice of n >= 3 nodes.  Validates the
 * constants (all positive, gamma > 1, rates in (0, 2)).  stream: see above.
 * No device memory is allocated.  The handle owns host state only. */
int lbm_init(lbm_handle** h, int64_t n, const lbm_params* p, void* stream);
void lbm_destroy(lbm_handle* h);
/* Changes the stream later calls enqueue on. */
int lbm_set_stream(lbm_handle* h, void* stream);
/* Replaces the constants (same validation as lbm_init). */
int lbm_set_params(lbm_handle* h, const lbm_params* p);

/* Workspace kinds. */
enum {
  LBM_WS_STEP = 0 /* lbm_step and lbm_diagnostics: a second state plus
                     reduction scratch */
};
/* Bytes of caller workspace that calls of the given kind need (0 on a bad
 * handle). */
size_t lbm_workspace_bytes(const lbm_handle* h, int kind);

/* Kernel selection.  lbm_set_tuning validates the shape (P in {2,4,8},
 * 1 <= K, 4K < 64P, waves_per_group in {1,2,4,8}). */
int lbm_set_tuning(lbm_handle* h, const lbm_tuning* t);
int lbm_get_tuning(const lbm_handle* h, lbm_tuning* t);

/* Equilibrium initialisation: f = M^-1 (rho, J, zeta, e_eq, psi_eq, eps_eq)
 * at every node, from device arrays rho, J, zeta of n doubles (the
 * equilibria of section 8, or of section 7 if eq_kind = 1).  f: device,
 * 6*n doubles. */
int lbm_set_equilibrium(lbm_handle* h, const double* rho, const double* J,
                        const double* zeta, double* f);

/* Advances the state f (device, 6*n doubles) by nsteps >= 0 time steps of the
 * algorithm of section 8, steps (i)-(viii), in place.  ws: device workspace
 * of lbm_workspace_bytes(h, LBM_WS_STEP) bytes, contents overwritten.
 * f and ws must not overlap. */
int lbm_step(lbm_handle* h, double* f, void* ws, size_t ws_bytes,
             int64_t nsteps);

/* Macroscopic moments of a state: m (device, 6*n doubles) = M f_d at every
 * node, in the order rho, J, zeta, e, psi, eps (eq. M-d1q3q3). */
int lbm_moments(lbm_handle* h, const double* f, double* m);

/* Diagnostics of a state (synchronising): out[0..7] = sum rho, sum J,
 * sum zeta, sum rho E, min rho, min T, count of non-finite entries of f,
 * count of nodes with rho <= 0 or T <= 0; rho E = p/(gamma-1) + J^2/(2 rho)
 * (section 5).  Returns LBM_ENONFINITE when either count is non-zero
 * (out is still filled). */
int lbm_diagnostics(lbm_handle* h, const double* f, void* ws, size_t ws_bytes,
                    double out[8]);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
