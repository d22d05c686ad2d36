// HIP kernels and C ABI of the coupled D1Q3Q3 lattice Boltzmann scheme
// (Dubois, Graille & Lallemand, arXiv 1802.02369) for gfx950.
//
// Forward kernels:
//   k_step_plain   one time step per launch, one node per thread; the
//                  neighbours' u and T for the source term go through LDS.
//   k_step_tile    K time steps per launch.  Each 64-lane wavefront owns a
//                  tile of 64*P consecutive nodes (P per lane, contiguous)
//                  held in VGPRs for all K steps; neighbour values move
//                  between lanes with DPP wave shifts.  A step has radius 2
//                  (the source reads u, T at j+-1 of the node whose
//                  populations stream to j+-1), so a tile loads 2K halo
//                  nodes on each side and stores its 64P - 4K interior nodes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/lbm.h"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

using lbm::Consts;

// ------------------------------------------------------------ errors ----

namespace lbm {
thread_local std::string g_err;

int set_err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return LBM_OK;
  return set_err(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }
static bool valid_rate(double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; }

int make_consts(const lbm_params* p, Consts* c) {
  if (!p) return set_err(LBM_EINVAL, "params is NULL");
  if (!finite_pos(p->lambda) || !finite_pos(p->rho0) || !finite_pos(p->cp) ||
      !finite_pos(p->prandtl) || !finite_pos(p->c0))
    return set_err(LBM_EINVAL,
                   "lambda, rho0, cp, prandtl and c0 must be finite and > 0");
  if (!(std::isfinite(p->gamma) && p->gamma > 1.0))
    return set_err(LBM_EINVAL, "gamma must be finite and > 1");
  if (!std::isfinite(p->s0) || !std::isfinite(p->u0_lin) ||
      !std::isfinite(p->s0_lin))
    return set_err(LBM_EINVAL, "s0, u0_lin, s0_lin must be finite");
  if (!valid_rate(p->s_e) || !valid_rate(p->s_psi) || !valid_rate(p->s_eps))
    return set_err(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
  if (p->source_on != 0 && p->source_on != 1)
    return set_err(LBM_EINVAL, "source_on must be 0 or 1");
  if (p->eq_kind != 0 && p->eq_kind != 1)
    return set_err(LBM_EINVAL, "eq_kind must be 0 or 1");
  if (p->eq_kind == 1 && (p->lambda != 1.0 || p->cp != 1.0 || p->rho0 != 1.0))
    return set_err(LBM_EINVAL,
                   "linear equilibria are defined for lambda = cp = rho0 = 1");
  const double l = p->lambda, cp = p->cp, r0 = p->rho0, g = p->gamma;
  std::memset(c, 0, sizeof *c);
  c->rho0 = r0;
  c->irho0 = 1.0 / r0;
  c->mJ = r0 * l;
  c->me = r0 * l * l;
  c->mz = r0 * cp;
  c->mpsi = r0 * cp * l;
  c->meps = r0 * cp * l * l;
  c->gm1 = g - 1.0;
  c->gcp = g / cp;
  c->xs0 = -g * p->s0 / cp;
  c->r = cp * (g - 1.0) / g;
  const double p0 = r0 * p->c0 * p->c0 / g;
  c->T0 = p0 / (r0 * c->r);
  c->two_l2 = 2.0 * l * l;
  c->eps_c = 2.0 * cp * l * l / g;
  c->s_e = p->s_e;
  c->s_psi = p->s_psi;
  c->s_eps = p->s_eps;
  c->src_c = p->source_on ? 0.25 * (1.0 / p->s_e - 0.5) : 0.0;
  c->cPr = cp / p->prandtl;
  c->fa = 1.0 / (3.0 * r0);
  c->fb = 1.0 / (3.0 * r0 * l * l);
  c->fc = 1.0 / (2.0 * r0 * l);
  c->ga = 1.0 / (3.0 * r0 * cp);
  c->gb = 1.0 / (3.0 * r0 * cp * l * l);
  c->gc = 1.0 / (2.0 * r0 * cp * l);
  c->gamma = g;
  c->cp = cp;
  c->eq_kind = p->eq_kind;
  if (p->eq_kind == 1) {
    // Eq. equilibres-NS-linearise as printed (lambda = cp = rho0 = 1).
    const double u0 = p->u0_lin, s0 = p->s0_lin, c0 = p->c0;
    c->lin[0] = 3.0 * (1.0 - s0) * c0 * c0 - 3.0 * u0 * u0 - 2.0;
    c->lin[1] = 6.0 * u0;
    c->lin[2] = 3.0 * u0 * u0;
    c->lin[3] = -u0 * s0;
    c->lin[4] = s0;
    c->lin[5] = u0;
    c->lin[6] = -3.0 * (s0 * c0) * (s0 * c0) - 6.0 * s0 * u0 * u0 +
                3.0 * s0 * c0 * c0 + 2.0 - 2.0 * s0 - 2.0 / g;
    c->lin[7] = 6.0 * u0 * s0;
    c->lin[8] = 3.0 * (u0 * u0 + s0 * c0 * c0);
  }
  return LBM_OK;
}

}  // namespace lbm

// ----------------------------------------------------------- kernels ----

namespace {

constexpr int kPlainBlock = 256;
constexpr int kDiagBlock = 256;
constexpr int kDiagMaxBlocks = 1024;

__global__ __launch_bounds__(256) void k_equilibrium(
    Consts c, const double* __restrict__ rho, const double* __restrict__ J,
    const double* __restrict__ zeta, double* __restrict__ f, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double v[6];
  lbm::equilibrium(c, rho[j], J[j], zeta[j], v);
#pragma unroll
  for (int k = 0; k < 6; ++k) f[k * n + j] = v[k];
}

__global__ __launch_bounds__(256) void k_moments(Consts c,
                                                 const double* __restrict__ f,
                                                 double* __restrict__ m,
                                                 int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double f0 = f[j], fp = f[n + j], fm = f[2 * n + j];
  const double g0 = f[3 * n + j], gp = f[4 * n + j], gm = f[5 * n + j];
  const double sf = fp + fm, sg = gp + gm;
  m[j] = lbm::density(c, f0, fp, fm);
  m[n + j] = c.mJ * (fp - fm);
  m[2 * n + j] = c.mz * (g0 + sg);
  m[3 * n + j] = c.me * (sf - 2.0 * f0);
  m[4 * n + j] = c.mpsi * (gp - gm);
  m[5 * n + j] = c.meps * (sg - 2.0 * g0);
}

// One time step, one node per thread, push streaming.  Block b owns nodes
// [b*B, b*B + B); threads 0 and 1 also compute u, T of the two halo nodes.
__global__ __launch_bounds__(kPlainBlock) void k_step_plain(
    Consts c, const double* __restrict__ fin, double* __restrict__ fout,
    int64_t n) {
  __shared__ double su[kPlainBlock + 2], sT[kPlainBlock + 2];
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * kPlainBlock;
  const int64_t rem = n - b0;
  const int nloc = rem < kPlainBlock ? (int)rem : kPlainBlock;
  const int64_t j = b0 + tid;
  const bool act = tid < nloc;
  double f0 = 0, fp = 0, fm = 0, g0 = 0, gp = 0, gm = 0, u, T, rw = 0, w = 0;
  if (act) {
    f0 = fin[j];
    fp = fin[n + j];
    fm = fin[2 * n + j];
    g0 = fin[3 * n + j];
    gp = fin[4 * n + j];
    gm = fin[5 * n + j];
    lbm::collide_local(c, f0, fp, fm, g0, gp, gm, u, T, rw, w);
    su[tid + 1] = u;
    sT[tid + 1] = T;
  }
  if (tid < 2) {
    const int64_t h = tid == 0 ? (b0 == 0 ? n - 1 : b0 - 1)
                               : (b0 + nloc == n ? 0 : b0 + nloc);
    double hu, hT;
    lbm::node_uT(c, fin[h], fin[n + h], fin[2 * n + h], fin[3 * n + h],
                 fin[4 * n + h], fin[5 * n + h], hu, hT);
    const int slot = tid == 0 ? 0 : nloc + 1;
    su[slot] = hu;
    sT[slot] = hT;
  }
  __syncthreads();
  if (!act) return;
  const double add = lbm::source_g(c, rw, w, su[tid], su[tid + 2], sT[tid],
                                   sT[tid + 2]);
  g0 += add;
  gp += add;
  gm += add;
  const int64_t jr = j + 1 == n ? 0 : j + 1;
  const int64_t jl = j == 0 ? n - 1 : j - 1;
  fout[j] = f0;
  fout[n + jr] = fp;
  fout[2 * n + jl] = fm;
  fout[3 * n + j] = g0;
  fout[4 * n + jr] = gp;
  fout[5 * n + jl] = gm;
}

// K time steps of one register-resident tile per wavefront (see the file
// header).  Tile t stores nodes [t*OUT, t*OUT + OUT) with OUT = 64P - 4K and
// loads nodes [t*OUT - 2K, t*OUT + OUT + 2K) (periodic).
template <int P>
__global__ __launch_bounds__(256) void k_step_tile(Consts c,
                                                   const double* __restrict__ fin,
                                                   double* __restrict__ fout,
                                                   int64_t n, int K,
                                                   int64_t ntiles) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (tile >= ntiles) return;  // uniform over the wavefront
  constexpr int W = 64 * P;
  const int H = 2 * K;
  const int OUT = W - 2 * H;
  const int64_t start = tile * OUT - H;
  double f[6][P];
  const bool inside = start >= 0 && start + W <= n;
  if (inside) {
    const double* src = fin + start + lane * P;
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) f[q][k] = src[q * n + k];
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int64_t g = lbm::wrap_mod(start + lane * P + k, n);
#pragma unroll
      for (int q = 0; q < 6; ++q) f[q][k] = fin[q * n + g];
    }
  }
  for (int step = 0; step < K; ++step) {
    double u[P], T[P], rw[P], w[P];
#pragma unroll
    for (int k = 0; k < P; ++k)
      lbm::collide_local(c, f[0][k], f[1][k], f[2][k], f[3][k], f[4][k],
                         f[5][k], u[k], T[k], rw[k], w[k]);
    const double uL = lbm::from_left(u[P - 1]), TL = lbm::from_left(T[P - 1]);
    const double uR = lbm::from_right(u[0]), TR = lbm::from_right(T[0]);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const double ul = k == 0 ? uL : u[k - 1];
      const double tl = k == 0 ? TL : T[k - 1];
      const double ur = k == P - 1 ? uR : u[k + 1];
      const double tr = k == P - 1 ? TR : T[k + 1];
      const double add = lbm::source_g(c, rw[k], w[k], ul, ur, tl, tr);
      f[3][k] += add;
      f[4][k] += add;
      f[5][k] += add;
    }
    // (viii) streaming: + populations move one node right, - one node left.
    const double fpL = lbm::from_left(f[1][P - 1]);
    const double gpL = lbm::from_left(f[4][P - 1]);
    const double fmR = lbm::from_right(f[2][0]);
    const double gmR = lbm::from_right(f[5][0]);
#pragma unroll
    for (int k = P - 1; k > 0; --k) {
      f[1][k] = f[1][k - 1];
      f[4][k] = f[4][k - 1];
    }
    f[1][0] = fpL;
    f[4][0] = gpL;
#pragma unroll
    for (int k = 0; k < P - 1; ++k) {
      f[2][k] = f[2][k + 1];
      f[5][k] = f[5][k + 1];
    }
    f[2][P - 1] = fmR;
    f[5][P - 1] = gmR;
  }
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int i = lane * P + k;
    const int64_t g = start + i;
    if (i >= H && i < W - H && g < n) {
#pragma unroll
      for (int q = 0; q < 6; ++q) fout[q * n + g] = f[q][k];
    }
  }
}

struct DiagAcc {
  double v[8];
};

__device__ inline void diag_combine(double* a, const double* b) {
  a[0] += b[0];
  a[1] += b[1];
  a[2] += b[2];
  a[3] += b[3];
  a[4] = fmin(a[4], b[4]);
  a[5] = fmin(a[5], b[5]);
  a[6] += b[6];
  a[7] += b[7];
}

// Block partials of the diagnostics, fixed tree order (deterministic).
__global__ __launch_bounds__(kDiagBlock) void k_diag_partial(
    Consts c, const double* __restrict__ f, int64_t n,
    double* __restrict__ partial) {
  __shared__ double s[kDiagBlock][8];
  double a[8] = {0, 0, 0, 0, INFINITY, INFINITY, 0, 0};
  for (int64_t j = (int64_t)blockIdx.x * kDiagBlock + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kDiagBlock) {
    const double f0 = f[j], fp = f[n + j], fm = f[2 * n + j];
    const double g0 = f[3 * n + j], gp = f[4 * n + j], gm = f[5 * n + j];
    const double v[6] = {f0, fp, fm, g0, gp, gm};
    double nf = 0;
    for (int k = 0; k < 6; ++k) nf += isfinite(v[k]) ? 0.0 : 1.0;
    const double rho = lbm::density(c, f0, fp, fm);
    const double J = c.mJ * (fp - fm);
    const double zeta = c.mz * (g0 + (gp + gm));
    double u, s_, X, T;
    lbm::thermo(c, rho, J, zeta, u, s_, X, T);
    const double p = rho * c.r * T;
    const double b[8] = {rho, J, zeta, p / c.gm1 + 0.5 * J * u,
                         rho, T, nf, (rho > 0.0 && T > 0.0) ? 0.0 : 1.0};
    diag_combine(a, b);
  }
  for (int k = 0; k < 8; ++k) s[threadIdx.x][k] = a[k];
  __syncthreads();
  for (int w = kDiagBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) diag_combine(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 8) partial[blockIdx.x * 8 + threadIdx.x] = s[0][threadIdx.x];
}

__global__ __launch_bounds__(kDiagBlock) void k_diag_final(
    const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  __shared__ double s[kDiagBlock][8];
  double a[8] = {0, 0, 0, 0, INFINITY, INFINITY, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kDiagBlock)
    diag_combine(a, partial + 8 * b);
  for (int k = 0; k < 8; ++k) s[threadIdx.x][k] = a[k];
  __syncthreads();
  for (int w = kDiagBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) diag_combine(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 8) out[threadIdx.x] = s[0][threadIdx.x];
}

}  // namespace

// ----------------------------------------------------- launch helpers ---

namespace lbm {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int launch_equilibrium(const Consts& c, const double* rho, const double* J,
                       const double* zeta, double* f, int64_t n,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_equilibrium, dim3((unsigned)cdiv(n, 256)), dim3(256), 0,
                     s, c, rho, J, zeta, f, n);
  return hip_check(hipGetLastError(), "k_equilibrium");
}

int launch_step_plain(const Consts& c, const double* fin, double* fout,
                      int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_step_plain, dim3((unsigned)cdiv(n, kPlainBlock)),
                     dim3(kPlainBlock), 0, s, c, fin, fout, n);
  return hip_check(hipGetLastError(), "k_step_plain");
}

int64_t tile_out(int P, int K) { return 64 * P - 4 * K; }

int launch_step_tile(const Consts& c, const double* fin, double* fout,
                     int64_t n, int P, int K, int wpg, hipStream_t s) {
  const int64_t ntiles = cdiv(n, tile_out(P, K));
  const dim3 grid((unsigned)cdiv(ntiles, wpg)), block(64 * wpg);
  switch (P) {
    case 2:
      hipLaunchKernelGGL(k_step_tile<2>, grid, block, 0, s, c, fin, fout, n, K,
                         ntiles);
      break;
    case 4:
      hipLaunchKernelGGL(k_step_tile<4>, grid, block, 0, s, c, fin, fout, n, K,
                         ntiles);
      break;
    case 8:
      hipLaunchKernelGGL(k_step_tile<8>, grid, block, 0, s, c, fin, fout, n, K,
                         ntiles);
      break;
    default:
      return set_err(LBM_EINVAL, "nodes_per_lane must be 2, 4 or 8");
  }
  return hip_check(hipGetLastError(), "k_step_tile");
}

size_t diag_ws_doubles() { return (size_t)kDiagMaxBlocks * 8 + 8; }

int launch_diagnostics(const Consts& c, const double* f, int64_t n,
                       double* scratch, hipStream_t s) {
  const int nb = (int)std::min<int64_t>(kDiagMaxBlocks, cdiv(n, kDiagBlock));
  hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(kDiagBlock), 0, s, c, f, n,
                     scratch + 8);
  int rc = hip_check(hipGetLastError(), "k_diag_partial");
  if (rc) return rc;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagBlock), 0, s,
                     scratch + 8, nb, scratch);
  return hip_check(hipGetLastError(), "k_diag_final");
}

int launch_moments(const Consts& c, const double* f, double* m, int64_t n,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_moments, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s,
                     c, f, m, n);
  return hip_check(hipGetLastError(), "k_moments");
}

}  // namespace lbm
