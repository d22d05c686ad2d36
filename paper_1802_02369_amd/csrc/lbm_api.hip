// C ABI entry points for one periodic lattice (declared in include/lbm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

namespace lbm {

int check_tuning(const lbm_tuning* t) {
  if (!t) return set_err(LBM_EINVAL, "tuning is NULL");
  if (t->kernel < LBM_KERNEL_AUTO || t->kernel > LBM_KERNEL_BLOCKED)
    return set_err(LBM_EINVAL, "unknown kernel %d", t->kernel);
  if (t->kernel == LBM_KERNEL_PLAIN) return LBM_OK;
  const int P = t->nodes_per_lane, K = t->steps_per_launch;
  if (P != 1 && P != 2 && P != 4 && P != 8)
    return set_err(LBM_EINVAL, "nodes_per_lane must be 1, 2, 4 or 8 (got %d)", P);
  const int w = t->waves_per_group;
  if (w != 1 && w != 2 && w != 4 && w != 8)
    return set_err(LBM_EINVAL, "waves_per_group must be 1, 2, 4 or 8");
  if (P == 1 && w != 1)
    return set_err(LBM_EINVAL, "nodes_per_lane 1 needs waves_per_group 1");
  if (K < 1 || 4 * K >= tile_nodes(P, w))
    return set_err(LBM_EINVAL,
                   "steps_per_launch must satisfy 1 <= K < P (62 "
                   "waves_per_group + 2) / 4");
  return LBM_OK;
}

StepSplit split_steps(int64_t nsteps, int K) {
  StepSplit out;
  if (nsteps <= 0 || K < 1) return out;
  int64_t L = (nsteps + K - 1) / K;
  if ((L & 1) && nsteps > L) ++L;
  out.count = L;
  out.base = nsteps / L;
  out.extra = nsteps % L;
  return out;
}

std::vector<lbm_tuning> tuning_candidates() {
  std::vector<lbm_tuning> v;
  const int Ps[] = {2, 4, 8}, Ws[] = {2, 4, 8}, Ks[] = {8, 12, 16, 24, 32, 40};
  for (int P : Ps)
    for (int W : Ws)
      for (int K : Ks)
        if (16 * K <= tile_nodes(P, W)) v.push_back(lbm_tuning{LBM_KERNEL_BLOCKED, P, K, W});
  return v;
}

lbm_tuning default_tuning(int64_t len, int64_t total, int eq) {
  // tile shapes from the widest down, with the K that measured best for
  // each.  The kernels that select the equilibria per lattice (eq != 0)
  // need over 256 VGPRs at P = 8, i.e. one wavefront per SIMD, so they
  // start at P = 4.
  // Small problems are bound by the latency of each step's chain of
  // arithmetic, not by throughput: their one-wavefront tiles take K = 16
  // (fewer launches) rather than the width's best, and at most 16384 nodes
  // in all one node per lane (half the chain per step, four times the
  // lane-nodes, on a chip that is mostly idle anyway): measured 2.5 -> 3.5
  // GLUPS at n = 2048 and 10.0 -> 13.7 at 8192 (K = 12), even at 32768 and
  // behind P = 2 above.  K = 13 ran the n = 8192 forward 3 % and its
  // gradient 5 % faster than K = 12 (K = 10, 11: slower; 14: +8 %, +3 %).
  static const lbm_tuning shapes[] = {
      {LBM_KERNEL_BLOCKED, 8, 40, 4}, {LBM_KERNEL_BLOCKED, 4, 24, 4},
      {LBM_KERNEL_BLOCKED, 2, 16, 4}, {LBM_KERNEL_BLOCKED, 2, 16, 1}};
  const int count = 4;
  for (int i = eq == 0 ? 0 : 1; i < count; ++i) {
    const lbm_tuning& t = shapes[i];
    const int64_t width = tile_width(t), out = width - 4 * t.steps_per_launch;
    if (4 * width <= len && total >= 1024 * out) return t;
  }
  if (total <= 16384) return lbm_tuning{LBM_KERNEL_BLOCKED, 1, 13, 1};
  return shapes[count - 1];
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

}  // namespace lbm

using namespace lbm;

// ------------------------------------------------ linear stability --
//
// Frozen-coefficient (von Neumann) analysis of one time step about a
// uniform state: the source of step (vii) is quadratic in gradients and
// drops out of the linearisation, so a Fourier mode e^{ikj} of the six
// populations is multiplied by G(k) = D(k) C', with C' the Jacobian of the
// node collision (steps (ii)-(vi)) and D(k) the streaming (f+, g+ from
// j - 1: e^{-ik}; f-, g- from j + 1: e^{ik}).  C' comes from complex-step
// differentiation of the collision written here in plain host arithmetic
// (physical moments, the library's equation of state and equilibria), so
// its entries are exact to rounding.
namespace {

template <class T>
void collide_host(const Consts& c, const T f[6], T out[6]) {
  const T rho = c.rho0 * f[0] + c.rho0 * f[1] + c.rho0 * f[2];
  const T J = c.mJ * (f[1] - f[2]);
  const T e = c.me * (f[1] + f[2] - 2.0 * f[0]);
  const T zeta = c.mz * (f[3] + f[4] + f[5]);
  const T psi = c.mpsi * (f[4] - f[5]);
  const T eps = c.meps * (f[4] + f[5] - 2.0 * f[3]);
  const T u = J / rho, s = zeta / rho;
  const T X = c.gm1 * std::log(rho / c.rho0) + c.gcp * s + c.xs0;
  T e_eq, psi_eq, eps_eq;
  if (c.eq_kind == 0) {
    e_eq = 3.0 * (J * u + rho * c.r * c.T0 * std::exp(X)) - c.two_l2 * rho;
    psi_eq = zeta * u;
    eps_eq = c.eps_c * rho * X + e_eq * s;
  } else if (c.eq_kind == 2) {
    const T p = rho * c.r * c.T0 * std::exp(c.gm1 * std::log(rho / c.rho0));
    e_eq = 3.0 * (J * u + p) - c.two_l2 * rho;
    psi_eq = 0.0;
    eps_eq = 0.0;
  } else {
    e_eq = c.lin[0] * rho + c.lin[1] * J + c.lin[2] * zeta;
    psi_eq = c.lin[3] * rho + c.lin[4] * J + c.lin[5] * zeta;
    eps_eq = c.lin[6] * rho + c.lin[7] * J + c.lin[8] * zeta;
  }
  const T es = e + c.s_e * (e_eq - e);
  const T ps = psi + c.s_psi * (psi_eq - psi);
  const T xs = eps + c.s_eps * (eps_eq - eps);
  const T fr = c.fa * rho, fe = c.fb * es, fj = c.fc * J;
  out[0] = fr - fe;
  out[1] = 0.5 * fe + fr + fj;
  out[2] = 0.5 * fe + fr - fj;
  const T gz = c.ga * zeta, ge = c.gb * xs, gj = c.gc * ps;
  out[3] = gz - ge;
  out[4] = 0.5 * ge + gz + gj;
  out[5] = 0.5 * ge + gz - gj;
}

using cplx = std::complex<double>;

// Spectral radius of a 6x6 complex matrix: ||A^n||^(1/n) for n = 2^50 by
// repeated squaring, renormalised at each squaring (the polynomial factors
// of non-normal or repeated eigenvalues vanish at that n).
double spectral_radius(const cplx (&A0)[6][6]) {
  cplx A[6][6];
  std::copy(&A0[0][0], &A0[0][0] + 36, &A[0][0]);
  double logs = 0.0;  // log of the scale taken out, per unit exponent
  double inv_n = 1.0;
  for (int it = 0; it < 50; ++it) {
    double nrm = 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) nrm = std::max(nrm, std::abs(A[i][j]));
    if (nrm == 0.0) return 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) A[i][j] /= nrm;
    logs += std::log(nrm) * inv_n;
    cplx B[6][6] = {};
    for (int i = 0; i < 6; ++i)
      for (int k = 0; k < 6; ++k)
        for (int j = 0; j < 6; ++j) B[i][j] += A[i][k] * A[k][j];
    std::copy(&B[0][0], &B[0][0] + 36, &A[0][0]);
    inv_n *= 0.5;
  }
  double nrm = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) nrm = std::max(nrm, std::abs(A[i][j]));
  return std::exp(logs + (nrm > 0.0 ? std::log(nrm) * inv_n : -INFINITY));
}

}  // namespace

namespace {

// The time steps of lbm_step once its arguments are checked: ws holds the
// second state (6 n doubles), then the diagnostics scratch with the failure
// record of LBM_CHECK_FINITE.
int step_run(lbm_handle* h, double* f, double* ws, int64_t nsteps) {
  const int64_t n = h->n;
  const size_t sbytes = (size_t)(6 * n) * sizeof(double);
  double* a = f;
  double* b = ws;
  // failure record of LBM_CHECK_FINITE, after the diagnostics scratch
  const bool check = (h->p.flags & LBM_CHECK_FINITE) != 0;
  unsigned long long* rec = reinterpret_cast<unsigned long long*>(
      ws + 6 * n + check_record_double());
  int rc = check ? launch_check_reset(rec, h->stream) : LBM_OK;
  int64_t launches = 0, done = 0;
  if (h->tune.kernel == LBM_KERNEL_PLAIN) {
    for (int64_t t = 0; t < nsteps && !rc; ++t) {
      rc = launch_step_plain(h->c, a, b, n, h->stream);
      if (!rc && check) rc = launch_check_state(h->c, b, n, t + 1, rec, h->stream);
      std::swap(a, b);
      ++launches;
    }
  } else {
    // An even number of launches leaves the result in f without a copy.
    for (int k : split_steps(nsteps, h->tune.steps_per_launch)) {
      rc = launch_step_tile(h->c, a, b, n, h->tune.nodes_per_lane, k,
                            h->tune.waves_per_group, h->stream);
      done += k;
      if (!rc && check) rc = launch_check_state(h->c, b, n, done, rec, h->stream);
      if (rc) break;
      std::swap(a, b);
      ++launches;
    }
  }
  if (rc) return rc;
  if (launches & 1)
    rc = hip_check(hipMemcpyAsync(f, ws, sbytes, hipMemcpyDeviceToDevice,
                                  h->stream),
                   "hipMemcpyAsync");
  if (rc || !check) return rc;
  unsigned long long key = 0;
  if ((rc = read_check_record(rec, h->stream, &key))) return rc;
  if (key == ~0ull) return LBM_OK;
  const long long steps = (long long)(key >> 36);
  return set_err(LBM_ENONFINITE,
                 "non-finite or non-physical state (rho <= 0 or T <= 0) after "
                 "%lld%s time steps: first failing node %lld",
                 steps, steps == kCheckMaxSteps1 ? " or more" : "",
                 (long long)(key & ((1ull << 36) - 1)));
}

// Scratch of lbm_step_noalloc: the second state and the diagnostics scratch
// of a lattice of up to LBM_NOALLOC_MAX_NODES nodes, as one device array
// that every device the library runs on holds until the process ends.  Host
// code never uses its name as an address (on the host it names a stand-in):
// noalloc_scratch takes each device's own address from hipGetSymbolAddress
// once, with that device current.
constexpr size_t kNoAllocDoubles = (size_t)6 * LBM_NOALLOC_MAX_NODES + 8192 + 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(double** out) {
  int dev = 0;
  int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices)
    return set_err(LBM_ENOTSUP, "device %d beyond the %d the library tracks", dev,
                   kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                   "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_linear_stability(const lbm_params* p, double rho, double u, double s,
                         int32_t nk, double* max_amp) {
  if (!p || !max_amp) return set_err(LBM_EINVAL, "NULL argument");
  Consts c;
  int rc = make_consts(p, &c);
  if (rc) return rc;
  if (!(std::isfinite(rho) && rho > 0.0) || !std::isfinite(u) ||
      !std::isfinite(s))
    return set_err(LBM_EINVAL, "need a finite state with rho > 0");
  if (nk < 2 || nk > (1 << 20))
    return set_err(LBM_EINVAL, "nk must lie in 2 .. 2^20");
  // populations of the uniform state: the collision's fixed point
  double feq[6];
  {
    Consts ce = c;
    ce.s_e = ce.s_psi = ce.s_eps = 1.0;  // one full relaxation lands on it
    double f0[6];
    const double ir = 1.0 / (3.0 * c.rho0);
    f0[0] = f0[1] = f0[2] = rho * ir;
    f0[1] += 0.5 * rho * u / c.mJ;
    f0[2] -= 0.5 * rho * u / c.mJ;
    f0[3] = f0[4] = f0[5] = rho * s / (3.0 * c.mz);
    collide_host<double>(ce, f0, feq);
  }
  // Jacobian of the collision by complex steps
  const double h = 1e-30;
  double Jc[6][6];
  for (int q = 0; q < 6; ++q) {
    cplx x[6], y[6];
    for (int i = 0; i < 6; ++i) x[i] = feq[i];
    x[q] += cplx(0.0, h);
    collide_host<cplx>(c, x, y);
    for (int i = 0; i < 6; ++i) Jc[i][q] = y[i].imag() / h;
  }
  double worst = 0.0;
  for (int j = 0; j < nk; ++j) {
    const double k = M_PI * j / (nk - 1);
    const cplx dm = std::polar(1.0, -k), dp = std::polar(1.0, k);
    const cplx d[6] = {1.0, dm, dp, 1.0, dm, dp};
    cplx G[6][6];
    for (int r = 0; r < 6; ++r)
      for (int q = 0; q < 6; ++q) G[r][q] = d[r] * Jc[r][q];
    worst = std::max(worst, spectral_radius(G));
  }
  *max_amp = worst;
  if (worst > 1.0 + 1e-10)
    return set_err(LBM_EUNSTABLE,
                   "linearly unstable about this state: amplification %.12g",
                   worst);
  return LBM_OK;
}

int lbm_coupled_rates(double s_e, double gamma, double prandtl, double* s_psi,
                      double* s_eps, double* ds_psi_ds_e) {
  if (!s_psi || !s_eps)
    return set_err(LBM_EINVAL, "s_psi and s_eps must not be NULL");
  if (!(std::isfinite(s_e) && s_e > 0.0 && s_e < 2.0))
    return set_err(LBM_EINVAL, "s_e must lie in (0, 2)");
  if (!(std::isfinite(gamma) && gamma > 1.0) ||
      !(std::isfinite(prandtl) && prandtl > 0.0))
    return set_err(LBM_EINVAL, "gamma must be > 1 and prandtl > 0");
  const double k = 1.5 * gamma / prandtl;
  const double sigma_e = 1.0 / s_e - 0.5;
  const double sp = 1.0 / (k * sigma_e + 0.5);
  *s_psi = sp;
  *s_eps = 1.5;
  if (ds_psi_ds_e) *ds_psi_ds_e = k * (sp / s_e) * (sp / s_e);
  return LBM_OK;
}

int lbm_init(lbm_handle** h, int64_t n, const lbm_params* p, void* stream) {
  if (!h) return set_err(LBM_EINVAL, "handle pointer is NULL");
  *h = nullptr;
  if (n < 3) return set_err(LBM_EINVAL, "lattice needs n >= 3 nodes (got %lld)",
                            (long long)n);
  if (n > kMaxNodes)
    return set_err(LBM_EINVAL, "n = %lld exceeds 2^36 nodes", (long long)n);
  Consts c;
  int rc = make_consts(p, &c);
  if (rc) return rc;
  lbm_handle* x = new lbm_handle;
  x->n = n;
  x->p = *p;
  x->c = c;
  x->stream = (hipStream_t)stream;
  x->tune = default_tuning(n, n, p->eq_kind == 0 ? 0 : -1);
  x->tune_default = true;
  *h = x;
  return LBM_OK;
}

void lbm_destroy(lbm_handle* h) {
  if (!h) return;
  lbm_batch_destroy(h->one);
  delete h;
}

int lbm_set_stream(lbm_handle* h, void* stream) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  h->stream = (hipStream_t)stream;
  if (h->one) lbm_batch_set_stream(h->one, stream);
  return LBM_OK;
}

int lbm_set_params(lbm_handle* h, const lbm_params* p) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  Consts c;
  int rc = make_consts(p, &c);
  if (rc) return rc;
  h->p = *p;
  h->c = c;
  if (h->tune_default) h->tune = default_tuning(h->n, h->n, p->eq_kind == 0 ? 0 : -1);
  lbm_batch_destroy(h->one);  // rebuilt with the new constants when needed
  h->one = nullptr;
  return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_handle* h, int kind) {
  if (!h) return 0;
  if (kind == LBM_WS_STEP)
    return (size_t)(6 * h->n + (int64_t)diag_ws_doubles()) * sizeof(double);
  if (kind == LBM_WS_TUNE)
    return (size_t)(12 * h->n + (int64_t)diag_ws_doubles()) * sizeof(double);
  return 0;
}

int lbm_set_tuning(lbm_handle* h, const lbm_tuning* t) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  int rc = check_tuning(t);
  if (rc) return rc;
  h->tune = *t;
  h->tune_default = false;
  if (h->tune.kernel == LBM_KERNEL_AUTO) h->tune.kernel = LBM_KERNEL_BLOCKED;
  return LBM_OK;
}

int lbm_get_tuning(const lbm_handle* h, lbm_tuning* t) {
  if (!h || !t) return set_err(LBM_EINVAL, "NULL argument");
  *t = h->tune;
  return LBM_OK;
}

int lbm_set_equilibrium(lbm_handle* h, const double* rho, const double* J,
                        const double* zeta, double* f) {
  if (!h || !rho || !J || !zeta || !f)
    return set_err(LBM_EINVAL, "NULL argument");
  return launch_equilibrium(h->c, rho, J, zeta, f, h->n, h->stream);
}

int lbm_moments(lbm_handle* h, const double* f, double* m) {
  if (!h || !f || !m) return set_err(LBM_EINVAL, "NULL argument");
  if (overlaps(f, 48 * h->n, m, 48 * h->n))
    return set_err(LBM_EINVAL, "f and m overlap");
  return launch_moments(h->c, f, m, h->n, h->stream);
}

int lbm_step(lbm_handle* h, double* f, void* ws, size_t ws_bytes,
             int64_t nsteps) {
  if (!h || !f || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (nsteps < 0) return set_err(LBM_EINVAL, "nsteps must be >= 0");
  const int64_t n = h->n;
  const size_t sbytes = (size_t)(6 * n) * sizeof(double);
  if (ws_bytes < lbm_workspace_bytes(h, LBM_WS_STEP))
    return set_err(LBM_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes,
                   lbm_workspace_bytes(h, LBM_WS_STEP));
  if (((uintptr_t)f | (uintptr_t)ws) & 7)
    return set_err(LBM_EINVAL, "f and ws must be 8-byte aligned");
  if (overlaps(f, sbytes, ws, ws_bytes))
    return set_err(LBM_EINVAL, "f and ws overlap");
  if (nsteps == 0) return LBM_OK;
  return step_run(h, f, (double*)ws, nsteps);
}

int lbm_step_noalloc(lbm_handle* h, double* f, int64_t nsteps) {
  if (!h || !f) return set_err(LBM_EINVAL, "NULL argument");
  if (nsteps < 0) return set_err(LBM_EINVAL, "nsteps must be >= 0");
  if (h->n > LBM_NOALLOC_MAX_NODES)
    return set_err(LBM_EINVAL,
                   "lbm_step_noalloc: n = %lld exceeds LBM_NOALLOC_MAX_NODES = %d "
                   "(its scratch is a fixed device array); use lbm_step with a "
                   "workspace", (long long)h->n, (int)LBM_NOALLOC_MAX_NODES);
  if ((uintptr_t)f & 7) return set_err(LBM_EINVAL, "f must be 8-byte aligned");
  double* ws = nullptr;
  int rc = noalloc_scratch(&ws);
  if (rc) return rc;
  if (overlaps(f, (size_t)(6 * h->n) * sizeof(double), ws,
               kNoAllocDoubles * sizeof(double)))
    return set_err(LBM_EINVAL, "f overlaps the library's scratch");
  if (nsteps == 0) return LBM_OK;
  return step_run(h, f, ws, nsteps);
}

int lbm_diagnostics(lbm_handle* h, const double* f, void* ws, size_t ws_bytes,
                    double out[8]) {
  if (!h || !f || !ws || !out) return set_err(LBM_EINVAL, "NULL argument");
  if (ws_bytes < lbm_workspace_bytes(h, LBM_WS_STEP))
    return set_err(LBM_EWORKSPACE, "workspace too small");
  double* scratch = (double*)ws + 6 * h->n;
  int rc = launch_diagnostics(h->c, f, h->n, scratch, h->stream);
  if (rc) return rc;
  rc = hip_check(hipMemcpyAsync(out, scratch, 8 * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream),
                 "hipMemcpyAsync");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  if (out[6] > 0 || out[7] > 0)
    return set_err(LBM_ENONFINITE,
                   "state holds %g non-finite values and %g nodes with rho<=0 "
                   "or T<=0",
                   out[6], out[7]);
  return LBM_OK;
}

}  // extern "C"
