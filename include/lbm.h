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

/* Functions of this header are the library's only exported symbols (it is
 * built with hidden visibility). */
#define LBM_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad pointer, size, constant or rate */
  LBM_EHIP = -2,       /* a HIP runtime call failed */
  LBM_EWORKSPACE = -3, /* workspace too small */
  LBM_ENONFINITE = -4, /* state holds NaN/Inf, rho <= 0 or T <= 0 */
  LBM_ENOTSUP = -5,    /* option not supported by this build */
  LBM_EUNSTABLE = -6   /* lbm_linear_stability: a Fourier mode grows */
};

/* Bits of lbm_params.flags. */
enum {
  /* Failure detection (opt-in).  lbm_step and lbm_batch_run check the state
   * at the end of every launch: a node fails when one of its six populations
   * is NaN or infinite, or its rho <= 0 or T <= 0 (T from the equation of
   * state, as lbm_diagnostics computes it).  The call then synchronises its
   * stream and returns LBM_ENONFINITE; lbm_last_error() names the number of
   * time steps done when the first failing launch ended and the lowest
   * failing node (single lattice) or lattice (batch) of that launch.  The
   * state is left as the run made it.  Each launch of K steps costs one more
   * pass over the state it wrote (48 bytes per node read); without the flag
   * nothing is checked and nothing waits. */
  LBM_CHECK_FINITE = 1
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
 *           (eq_kind = 1); u0_lin is also the advection velocity u0 of the
 *           thermal scheme (eq_kind = 3)
 *   alpha   eps_eq = alpha lambda^2 zeta of the thermal scheme (eq_kind = 3),
 *           -2 < alpha < 1 (section 4)
 *   source_on  1: add the entropy production of step (vii) of section 8
 *   eq_kind    0: nonlinear equilibria of section 8 (eqs. energie-equilibre,
 *              psi-equilibre, eq-energie-entropie-d1q3q3);
 *              1: linear equilibria of section 7 (eq. equilibres-NS-linearise,
 *              printed for lambda = cp = rho0 = 1; other values are rejected),
 *              with the zeta coefficient of e_eq taken as 3 c0^2 / cp (the
 *              print shows 3 u0^2 / cp; the zeta term of the J flux in eq.
 *              NS-rho-J-zeta-linearise requires c0^2);
 *              2: fluid D1Q3 scheme of sections 2-3 (eq. energie-equilibre
 *              with the isentropic pressure p0 (rho/rho0)^gamma), the g
 *              distribution passive (psi_eq = eps_eq = 0);
 *              3: thermal D1Q3 advection-diffusion scheme of section 4
 *              (psi_eq = u0 zeta, eps_eq = alpha lambda^2 zeta), the f
 *              distribution passive (e_eq = (3 c0^2 - 2 lambda^2) rho).
 *              Kinds 2 and 3 need source_on = 0.
 *   flags      LBM_CHECK_FINITE or 0 (other bits: LBM_EINVAL); in a batch,
 *              the lattices whose flags have it are checked
 *   reserved   must be 0
 */
typedef struct lbm_params {
  double lambda, rho0, cp, gamma, prandtl, c0, s0;
  double s_e, s_psi, s_eps;
  double u0_lin, s0_lin;
  double alpha;
  int32_t source_on;
  int32_t eq_kind;
  int32_t flags;
  int32_t reserved;
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
  int32_t waves_per_group; /* wavefronts per tile (blocked kernel) */
} lbm_tuning;

/* ----------------------------------------------------------------- misc */

/* Message of the last failing call on this thread ("" if none). */
LBM_API const char* lbm_last_error(void);

/* Relaxation coupling of section 7: sigma = 1/s - 1/2 (eq. henon),
 * sigma_psi = (3/2)(gamma/Pr) sigma_e (eq. lien-sigma-sigma), s_eps = 1.5
 * (step (iii) of section 8).  ds_psi_ds_e (may be NULL) receives the
 * derivative of s_psi with respect to s_e.  Host only. */
LBM_API int lbm_coupled_rates(double s_e, double gamma, double prandtl, double* s_psi,
                              double* s_eps, double* ds_psi_ds_e);

/* Opt-in check of the rates against linear stability (the analysis of
 * section 7, with the coupled equilibria of section 8): the largest modulus
 * *max_amp, over the Fourier modes k = pi j / (nk - 1), j = 0 .. nk - 1, of
 * the eigenvalues of one time step's amplification matrix about the
 * uniform state rho, u, s (physical units; the source is quadratic in
 * gradients and drops out).  Returns LBM_EUNSTABLE when it exceeds
 * 1 + 1e-10 (a mode grows: the scheme about such a state diverges),
 * LBM_OK otherwise, LBM_EINVAL for bad constants, rho <= 0 or nk outside
 * 2 .. 2^20.  Host only; nothing else calls it. */
LBM_API int lbm_linear_stability(const lbm_params* p, double rho, double u,
                                 double s, int32_t nk, double* max_amp);

/* ----------------------------------------------------- single lattice */

/* Creates a handle for one periodic lattice of 3 <= n <= 2^36 nodes.  Validates the
 * constants (all positive, gamma > 1, rates in (0, 2)).  stream: see above.
 * No device memory is allocated.  The handle owns host state only. */
LBM_API int lbm_init(lbm_handle** h, int64_t n, const lbm_params* p, void* stream);
LBM_API void lbm_destroy(lbm_handle* h);
/* Changes the stream later calls enqueue on. */
LBM_API int lbm_set_stream(lbm_handle* h, void* stream);
/* Replaces the constants (same validation as lbm_init). */
LBM_API int lbm_set_params(lbm_handle* h, const lbm_params* p);

/* Workspace kinds. */
enum {
  LBM_WS_STEP = 0, /* lbm_step, lbm_diagnostics (and the batch forms): a
                      second state plus tables and reduction scratch */
  LBM_WS_TUNE = 1  /* lbm_autotune / lbm_batch_autotune: LBM_WS_STEP for
                      every candidate shape plus a copy of the state */
};
/* Bytes of caller workspace that calls of the given kind need (0 on a bad
 * handle). */
LBM_API size_t lbm_workspace_bytes(const lbm_handle* h, int kind);

/* Kernel selection.  lbm_set_tuning validates the shape (P in {1,2,4,8},
 * waves_per_group W in {1,2,4,8}, W = 1 when P = 1, 1 <= K,
 * 4K < P (62 W + 2), i.e. K <= 15 at P = 1).
 * The blocked kernel gives each workgroup of W wavefronts a tile of
 * P (62 W + 2) nodes held in registers for K steps (64 P per wavefront,
 * neighbouring wavefronts sharing two lanes; 64 nodes at P = 1) and stores
 * its interior of P (62 W + 2) - 4K nodes.  The
 * default depends on the lattice length and the equilibria: for eq_kind 0,
 * P = 8, K = 40, 4 wavefronts for long lattices; for eq_kind 1 or 2 (kernels
 * that select the equilibria per lattice and need more registers at P = 8)
 * P = 4, K = 24, 4 wavefronts; narrower tiles for short lattices or few
 * tiles, down to P = 1, K = 13 for problems of at most 16384 nodes in all
 * (bound by the latency of each step rather than by throughput).
 * lbm_set_params re-derives the default unless lbm_set_tuning or
 * lbm_autotune chose the shape.  Every
 * kernel and tile shape rounds each node-update identically: results are
 * bitwise independent of the tuning. */
LBM_API int lbm_set_tuning(lbm_handle* h, const lbm_tuning* t);
LBM_API int lbm_get_tuning(const lbm_handle* h, lbm_tuning* t);

/* Equilibrium initialisation: f = M^-1 (rho, J, zeta, e_eq, psi_eq, eps_eq)
 * at every node, from device arrays rho, J, zeta of n doubles (the
 * equilibria of section 8, or of section 7 if eq_kind = 1).  f: device,
 * 6*n doubles. */
LBM_API int lbm_set_equilibrium(lbm_handle* h, const double* rho, const double* J,
                                const double* zeta, double* f);

/* Advances the state f (device, 6*n doubles) by nsteps >= 0 time steps of the
 * algorithm of section 8, steps (i)-(viii), in place.  ws: device workspace
 * of lbm_workspace_bytes(h, LBM_WS_STEP) bytes, contents overwritten.
 * f and ws must not overlap.  With LBM_CHECK_FINITE in the lattice's flags
 * the call checks the state after every launch, synchronises and returns
 * LBM_ENONFINITE if a node failed (see LBM_CHECK_FINITE; the step count in
 * the message saturates at 2^28 - 1). */
LBM_API int lbm_step(lbm_handle* h, double* f, void* ws, size_t ws_bytes,
                     int64_t nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_step
 * without a workspace argument.  The second state and the reduction scratch
 * live in one fixed device array of the library, of
 * 8 (6 LBM_NOALLOC_MAX_NODES + 8256) bytes (about 48 MiB), which each device
 * the library runs on holds until the process ends; the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).  Lattices of
 * more than LBM_NOALLOC_MAX_NODES nodes are rejected with LBM_EINVAL.  All
 * calls on one device share that array: calls that overlap in time on one
 * device (other threads, other streams, or kernels still running from an
 * earlier call on another stream) race and give wrong results; calls on one
 * stream are ordered and safe.  The array keeps the last call's contents;
 * nothing in it needs to start at zero (each launch writes every node of
 * the state it produces, and the failure record of LBM_CHECK_FINITE is reset
 * by a kernel at the start of each call).  Otherwise as lbm_step, with the
 * same results bitwise. */
#define LBM_NOALLOC_MAX_NODES (1 << 20)
LBM_API int lbm_step_noalloc(lbm_handle* h, double* f, int64_t nsteps);

/* Macroscopic moments of a state: m (device, 6*n doubles) = M f_d at every
 * node, in the order rho, J, zeta, e, psi, eps (eq. M-d1q3q3). */
LBM_API int lbm_moments(lbm_handle* h, const double* f, double* m);

/* Diagnostics of a state (synchronising): out[0..7] = sum rho, sum J,
 * sum zeta, sum rho E, min rho, min T, count of non-finite entries of f,
 * count of nodes with rho <= 0 or T <= 0; rho E = p/(gamma-1) + J^2/(2 rho)
 * (section 5).  Returns LBM_ENONFINITE when either count is non-zero
 * (out is still filled). */
LBM_API int lbm_diagnostics(lbm_handle* h, const double* f, void* ws, size_t ws_bytes,
                            double out[8]);

/* Autotuner (synchronising).  Times the blocked kernel on the caller's state
 * f with each candidate shape (P in {2,4,8}, waves per tile in {2,4,8}, K in
 * {8,12,16,24,32,40}, halo recomputation at most a quarter of the tile) for
 * probe_steps time steps rounded up to a multiple of 2K (so that every launch
 * runs the candidate's own K), plus the one-step kernel for probe_steps,
 * keeps the fastest per step, and restores f.  ws: lbm_workspace_bytes(h, LBM_WS_TUNE) bytes.  cache_path
 * (may be NULL) names a JSON file mapping "<gfx arch>/<kind>/<size class>/
 * <equilibrium class>/<kernel generation>" to the chosen shape; a hit skips
 * the timing, a miss adds the entry.  The
 * chosen shape becomes the handle's tuning and is returned in *out (may be
 * NULL). */
LBM_API int lbm_autotune(lbm_handle* h, double* f, void* ws, size_t ws_bytes,
                         int64_t probe_steps, const char* cache_path, lbm_tuning* out);

/* ----------------------------------------------- gradients (reverse mode)
 *
 * Gradients of a final-time loss through nsteps time steps: the forward run
 * keeps the state every ckpt_every steps (about sqrt(nsteps) is the usual
 * choice), the reverse sweep recomputes each segment from its checkpoint and
 * runs the adjoint of the step (streaming, collision, source) backwards.  The
 * relaxation rates s_e, s_psi, s_eps are independent inputs here (s_e also
 * sets the viscosity of the source term); a caller that couples s_psi to s_e
 * (lbm_coupled_rates) applies d s_psi / d s_e itself. */

/* Bytes of the workspace that lbm_forward_ckpt / lbm_adjoint / lbm_loss /
 * lbm_equilibrium_adjoint / lbm_moments_adjoint use for this nsteps and
 * ckpt_every with the current tile shape, reverse kernel and recompute
 * stride (0 on bad arguments): ceil(nsteps/ckpt_every) checkpoints, the
 * stored recomputed states (m = min(ckpt_every, nsteps) - 1 of them, or
 * floor(m/2) at stride 2, see lbm_set_recompute_stride), one more state and
 * tables.  The recomputed states are held twice when the reverse sweep is
 * pipelined: with the blocked reverse kernel on problems whose reverse
 * launches hold fewer than 2048 wavefronts (small lattices), the recompute
 * of one checkpoint segment runs on a second stream beside the reverse
 * steps of the next. */
LBM_API size_t lbm_adjoint_workspace_bytes(lbm_handle* h, int64_t nsteps,
                                           int64_t ckpt_every);
/* Advances f (device, 6*n) by nsteps steps in place like lbm_step, keeping
 * the checkpoints in ws.  Required before the calls below with the same ws,
 * nsteps and ckpt_every. */
LBM_API int lbm_forward_ckpt(lbm_handle* h, double* f, void* ws, size_t ws_bytes,
                             int64_t nsteps, int64_t ckpt_every);
/* Reverse sweep (synchronising for rbar).  fbar (device, 6*n): on entry
 * dL/df(T), on return dL/df(0).  rbar (host, 3): dL/d(s_e, s_psi, s_eps).
 * use_graph = 1 captures the launch sequence into a hipGraph on first use
 * (re-captured when ws, nsteps, ckpt_every, fbar or the tuning change). */
LBM_API int lbm_adjoint(lbm_handle* h, void* ws, size_t ws_bytes, int64_t nsteps,
                        int64_t ckpt_every, double* fbar, double rbar[3],
                        int use_graph);
/* L = 1/2 sum_j (rho_j - target_j)^2 of the state f (target: device n
 * doubles, or NULL for rho0 everywhere); *loss (host, synchronising) and
 * fbar = dL/df (device, 6*n). */
LBM_API int lbm_loss(lbm_handle* h, const double* f, const double* target, void* ws,
                     size_t ws_bytes, double* loss, double* fbar);
/* Reverse of lbm_set_equilibrium: given fbar = dL/df(0), the adjoints of the
 * initial fields (device, n doubles each). */
LBM_API int lbm_equilibrium_adjoint(lbm_handle* h, const double* rho, const double* J,
                                    const double* zeta, const double* fbar,
                                    double* rho_bar, double* J_bar, double* zeta_bar,
                                    void* ws, size_t ws_bytes);
/* Reverse of lbm_moments: fbar = M^T mbar (device, 6*n each). */
LBM_API int lbm_moments_adjoint(lbm_handle* h, const double* mbar, double* fbar,
                                void* ws, size_t ws_bytes);
/* Kernel of the reverse sweep.  LBM_KERNEL_BLOCKED keeps dL/df in registers
 * for up to K reverse steps of a tile of P (62 W + 2) nodes, neighbouring
 * wavefronts sharing two lanes that are refreshed through LDS before each
 * step (one workgroup barrier per step; P = 2 with W the forward's
 * wavefronts, or P W / 2 for P = 4, 8, at most 4; P = 1, W = 1 after a
 * forward at P = 1; halo 2K, or 2K + 2 at recompute stride 2), reading only
 * the stored recomputed forward states, the next one prefetched while the
 * current step computes (about 2.4x the arithmetic of a forward step per
 * node-step).  LBM_KERNEL_PLAIN runs one reverse step per launch, one node
 * per thread (HBM-bound, 144 B per node-step).  LBM_KERNEL_AUTO (the
 * default) takes the blocked kernel wherever its tiles can hold the halo,
 * else the one-step kernel.  A halo too wide for P = 2 tiles
 * (4K >= 2 (62 W + 2)) falls back to P = 4 with 8 wavefronts; lbm_forward_ckpt
 * rejects with LBM_ENOTSUP an explicit LBM_KERNEL_BLOCKED whose halo leaves
 * even those no interior (4K >= 1992).  Takes effect at the next
 * lbm_forward_ckpt. */
LBM_API int lbm_set_adjoint_kernel(lbm_handle* h, int kernel);
/* Stride of the recomputed forward states that the blocked reverse sweep
 * stores: 1 keeps every state of a checkpoint segment; 2 keeps the even ones
 * only, and the reverse kernel recomputes each odd state from the one before
 * (one forward step per two reverse steps, bitwise the stored value) in
 * place of a store and a load of 48 bytes per node, with half the segment
 * buffer and a halo of 2K + 2.  0 (the default) takes 2 where the reverse
 * launches hold at least 2048 wavefronts (large problems, whose sweep is
 * bound by those loads and stores) and 1 elsewhere.  Stride 2 applies only
 * to the blocked kernel at P = 2 with K >= 2 (elsewhere the sweep keeps
 * every state).  Results do not depend on it.  Takes effect at the next
 * lbm_forward_ckpt; LBM_EINVAL for a stride outside 0..2. */
LBM_API int lbm_set_recompute_stride(lbm_handle* h, int stride);

/* ------------------------------------------------- batches of lattices */

/* A batch of n_inst independent periodic lattices of different lengths and
 * constants, advanced together (the paper runs one lattice at a time; the
 * batch is a throughput form of the same algorithm, lattice by lattice).
 * offsets (host, n_inst+1 int64, offsets[0] = 0, lengths offsets[i+1] -
 * offsets[i] >= 3) place lattice i at [offsets[i], offsets[i+1]) of every
 * array of a batch state of 6 * n_total doubles, n_total = offsets[n_inst]
 * (array k of the state is doubles [k*n_total, (k+1)*n_total)).  params
 * (host, n_inst records) are validated as in lbm_init.  Both are copied. */
LBM_API int lbm_batch_init(lbm_batch** b, int64_t n_inst, const int64_t* offsets,
                           const lbm_params* params, void* stream);
LBM_API void lbm_batch_destroy(lbm_batch* b);
LBM_API int lbm_batch_set_stream(lbm_batch* b, void* stream);
/* Tile shape of the batch (as lbm_set_tuning; the blocked kernel only).
 * Clears any shape groups. */
LBM_API int lbm_batch_set_tuning(lbm_batch* b, const lbm_tuning* t);
LBM_API int lbm_batch_get_tuning(const lbm_batch* b, lbm_tuning* t);

/* Shape groups of lbm_batch_run.  A tile holds nodes of one lattice, so a
 * lattice of L nodes costs ceil(L / (P (62 W + 2) - 4K)) tiles, the last of
 * them (or the only one, for a lattice shorter than a tile) running just the
 * wavefronts its nodes and halos need: short lattices still waste part of a
 * wide tile, long ones run best on it.  With
 * groups, lattice i runs with shapes[group_of[i]] (host arrays of n_groups
 * and n_inst entries, 1 <= n_groups <= LBM_MAX_GROUPS), each group as its
 * own sequence of launches on its own stream, forked from the batch's
 * stream and joined back to it (also inside the graph of use_graph = 1).
 * Results are bitwise those of a single shape.  n_groups = 0 returns to the
 * single tuning.  Takes effect at the next lbm_batch_prepare; the adjoint
 * calls keep using the single tuning.  lbm_batch_autotune sets groups when
 * they time faster. */
enum { LBM_MAX_GROUPS = 4 };
LBM_API int lbm_batch_set_groups(lbm_batch* b, int32_t n_groups,
                                 const lbm_tuning* shapes, const int32_t* group_of);
/* *n_groups (0: single tuning); shapes (capacity LBM_MAX_GROUPS) and
 * group_of (capacity n_inst) receive the assignment unless NULL. */
LBM_API int lbm_batch_get_groups(const lbm_batch* b, int32_t* n_groups,
                                 lbm_tuning* shapes, int32_t* group_of);
/* Resident lattices of lbm_batch_run.  With mode 1 (the default) every
 * lattice of LBM_RESIDENT_MIN..LBM_RESIDENT_MAX nodes runs all nsteps steps
 * inside one launch (up to 65536 steps per launch): its state is loaded once
 * into registers (8 nodes per lane, one wavefront per 496 nodes, lattices
 * packed into workgroups of 12 wavefronts), advanced step after step with
 * the periodic wrap and the neighbouring wavefronts' edge nodes exchanged
 * through LDS every 4 steps, and stored once (96 bytes of HBM per node for
 * the whole run).  That launch
 * runs on a side stream of the batch, forked from its stream and joined back
 * to it (also inside the graph of use_graph = 1), beside the tiled launches
 * of the other lattices; shape groups apply to those only.  Mode 0 runs
 * every lattice in tiles.  Results are bitwise the same in both modes.
 * lbm_batch_autotune, called in mode 1, also times mode 0 and keeps the
 * faster (a batch of short lattices only can fill the chip better with
 * tiles).  Only batches whose lattices all have eq_kind 0 run lattices
 * resident.  Takes effect at the next lbm_batch_prepare; the adjoint calls
 * always use tiles.  LBM_EINVAL for another mode. */
enum { LBM_RESIDENT_MIN = 16, LBM_RESIDENT_MAX = 5952 };
LBM_API int lbm_batch_set_resident(lbm_batch* b, int mode);
/* Number of lattices that run resident with the current mode. */
LBM_API int64_t lbm_batch_resident_lattices(const lbm_batch* b);
/* Total nodes n_total of the batch (0 on a bad handle). */
LBM_API int64_t lbm_batch_total_nodes(const lbm_batch* b);
LBM_API size_t lbm_batch_workspace_bytes(const lbm_batch* b, int kind);
/* Uploads the per-lattice constants, offsets and the tile table of the
 * current tuning into ws (synchronising).  Required before the calls below
 * whenever ws, the tuning or the constants change. */
LBM_API int lbm_batch_prepare(lbm_batch* b, void* ws, size_t ws_bytes);
/* Equilibrium initialisation of every lattice from device arrays rho, J,
 * zeta of n_total doubles (batch layout). */
LBM_API int lbm_batch_set_equilibrium(lbm_batch* b, const double* rho, const double* J,
                                      const double* zeta, double* f, void* ws,
                                      size_t ws_bytes);
/* Advances every lattice of the batch state f (device, 6*n_total doubles) by
 * nsteps time steps, in place.  With use_graph = 1 the launches are captured
 * once into a hipGraph (re-captured when f, ws, nsteps or the tuning change)
 * and replayed with one hipGraphLaunch on the stream.  Lattices with
 * LBM_CHECK_FINITE in their flags are checked after every launch (the
 * checks and the reset of the failure record are kernels inside the graph);
 * if any has them, the call synchronises and returns LBM_ENONFINITE when one
 * failed, naming the step count and the lowest lattice index (saturating at
 * 2^32 - 1 steps). */
LBM_API int lbm_batch_run(lbm_batch* b, double* f, void* ws, size_t ws_bytes,
                          int64_t nsteps, int use_graph);
/* Moments m = M f of every node (device, 6*n_total doubles, moment order as
 * lbm_moments). */
LBM_API int lbm_batch_moments(lbm_batch* b, const double* f, double* m, void* ws,
                              size_t ws_bytes);
/* Per-lattice diagnostics (synchronising): out (host, 8*n_inst doubles) gets
 * the eight values of lbm_diagnostics for each lattice.  Returns
 * LBM_ENONFINITE if any lattice has a non-finite or non-physical node. */
LBM_API int lbm_batch_diagnostics(lbm_batch* b, const double* f, void* ws,
                                  size_t ws_bytes, double* out);
/* Autotuner of the batch (as lbm_autotune; calls lbm_batch_prepare): the
 * tile shape, shape groups, and in resident mode 1 the mode itself. */
LBM_API int lbm_batch_autotune(lbm_batch* b, double* f, void* ws, size_t ws_bytes,
                               int64_t probe_steps, const char* cache_path,
                               lbm_tuning* out);

/* Batch forms of the gradient calls: as above, lattice by lattice.  rbar
 * (device, 3*n_inst) holds dL_i/d(s_e, s_psi, s_eps) of lattice i; loss
 * (device, n_inst) the per-lattice losses.  Rate gradients are reduced in a
 * fixed order (deterministic). */
LBM_API size_t lbm_batch_adjoint_workspace_bytes(const lbm_batch* b, int64_t nsteps,
                                                 int64_t ckpt_every);
LBM_API int lbm_batch_forward_ckpt(lbm_batch* b, double* f, void* ws, size_t ws_bytes,
                                   int64_t nsteps, int64_t ckpt_every);
LBM_API int lbm_batch_adjoint(lbm_batch* b, void* ws, size_t ws_bytes, int64_t nsteps,
                              int64_t ckpt_every, double* fbar, double* rbar,
                              int use_graph);
LBM_API int lbm_batch_loss(lbm_batch* b, const double* f, const double* target,
                           void* ws, size_t ws_bytes, double* loss, double* fbar);
LBM_API int lbm_batch_equilibrium_adjoint(lbm_batch* b, const double* rho,
                                          const double* J, const double* zeta,
                                          const double* fbar, double* rho_bar,
                                          double* J_bar, double* zeta_bar, void* ws,
                                          size_t ws_bytes);
LBM_API int lbm_batch_moments_adjoint(lbm_batch* b, const double* mbar, double* fbar,
                                      void* ws, size_t ws_bytes);
LBM_API int lbm_batch_set_adjoint_kernel(lbm_batch* b, int kernel);
LBM_API int lbm_batch_set_recompute_stride(lbm_batch* b, int stride);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
