// HIP kernels and C ABI of the coupled D1Q3Q3 lattice Boltzmann scheme
// (Dubois, Graille & Lallemand, arXiv 1802.02369) for gfx950.
//
// Forward kernels:
//   k_step_plain   one time step per launch, one node per thread; the
//                  neighbours' u and T for the source term and the streamed
//                  populations go through LDS, so every store is aligned.
//   k_step_tile    K time steps per launch.  Each 64-lane wavefront holds
//                  64*P consecutive nodes (P per lane, contiguous) in VGPRs
//                  for all K steps; neighbour values move between lanes with
//                  DPP wave shifts, and the wavefronts of a workgroup overlap
//                  by two lanes that are refreshed through LDS every P/2
//                  steps.  A step has radius 2 (the source reads u, T at
//                  j+-1 of the node whose populations stream to j+-1), so a
//                  tile loads 2K halo nodes on each side and stores its
//                  interior.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>

#include "../../include/lbm.h"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_tile.hpp"

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
      !std::isfinite(p->s0_lin) || !std::isfinite(p->alpha))
    return set_err(LBM_EINVAL, "s0, u0_lin, s0_lin, alpha must be finite");
  if (!valid_rate(p->s_e) || !valid_rate(p->s_psi) || !valid_rate(p->s_eps))
    return set_err(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
  if (p->source_on != 0 && p->source_on != 1)
    return set_err(LBM_EINVAL, "source_on must be 0 or 1");
  if (p->eq_kind < 0 || p->eq_kind > 3)
    return set_err(LBM_EINVAL, "eq_kind must be 0, 1, 2 or 3");
  if (p->eq_kind >= 2 && p->source_on)
    return set_err(LBM_EINVAL, "the single-distribution schemes need source_on = 0");
  if (p->eq_kind == 3 && !(p->alpha > -2.0 && p->alpha < 1.0))
    return set_err(LBM_EINVAL, "alpha must lie in (-2, 1)");
  if (p->eq_kind == 1 && (p->lambda != 1.0 || p->cp != 1.0 || p->rho0 != 1.0))
    return set_err(LBM_EINVAL,
                   "linear equilibria are defined for lambda = cp = rho0 = 1");
  if ((p->flags & ~LBM_CHECK_FINITE) != 0 || p->reserved != 0)
    return set_err(LBM_EINVAL, "flags may hold LBM_CHECK_FINITE only; reserved must be 0");
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
  c->se_2 = p->s_e / 2.0;
  c->ise2 = 1.0 / (p->s_e * p->s_e);
  c->se_3 = p->s_e / 3.0;
  c->se_6 = p->s_e / 6.0;
  c->sp_2 = p->s_psi / 2.0;
  c->sx_3 = p->s_eps / 3.0;
  c->sx_6 = p->s_eps / 6.0;
  c->hP = p->c0 * p->c0 / (g * l * l);
  c->two_g = 2.0 / g;
  c->hS = c->src_c * l * l / (3.0 * cp * c->T0);
  c->hC = cp * c->T0 / (p->prandtl * l * l);
  c->hSd = p->source_on ? -0.25 * c->ise2 * l * l / (3.0 * cp * c->T0) : 0.0;
  c->xs0l = c->xs0 - c->gm1 * std::log(r0);
  c->eq_kind = p->eq_kind;
  c->flags = p->flags;
  if (p->eq_kind == 1) {
    // Eq. equilibres-NS-linearise (lambda = cp = rho0 = 1).  The zeta
    // coefficient of e_eq is 3 c0^2 (printed 3 u0^2): the flux of J in
    // eq. NS-rho-J-zeta-linearise has the term c0^2 d_x zeta, and the
    // printed psi_eq, eps_eq are compatible with that system's entropy
    // equation at second order only with it.
    const double u0 = p->u0_lin, s0 = p->s0_lin, c0 = p->c0;
    c->lin[0] = 3.0 * (1.0 - s0) * c0 * c0 - 3.0 * u0 * u0 - 2.0;
    c->lin[1] = 6.0 * u0;
    c->lin[2] = 3.0 * c0 * c0;
    c->lin[3] = -u0 * s0;
    c->lin[4] = s0;
    c->lin[5] = u0;
    c->lin[6] = -3.0 * (s0 * c0) * (s0 * c0) - 6.0 * s0 * u0 * u0 +
                3.0 * s0 * c0 * c0 + 2.0 - 2.0 * s0 - 2.0 / g;
    c->lin[7] = 6.0 * u0 * s0;
    c->lin[8] = 3.0 * (u0 * u0 + s0 * c0 * c0);
  } else if (p->eq_kind == 3) {
    // Thermal scheme of section 4: its equilibria are linear in (rho, J,
    // zeta), so it runs on the linear path.
    c->eq_kind = 1;
    c->lin[0] = 3.0 * p->c0 * p->c0 - 2.0 * l * l;
    c->lin[5] = p->u0_lin;
    c->lin[8] = p->alpha * l * l;
  }
  // the same linear equilibria in scaled moments: e / (rho0 lambda^2),
  // psi / (rho0 cp lambda), eps / (rho0 cp lambda^2) in terms of
  // rho / rho0, J / (rho0 lambda), zeta / (rho0 cp)
  c->hlin[0] = c->lin[0] / (l * l);
  c->hlin[1] = c->lin[1] / l;
  c->hlin[2] = c->lin[2] * cp / (l * l);
  c->hlin[3] = c->lin[3] / (cp * l);
  c->hlin[4] = c->lin[4] / cp;
  c->hlin[5] = c->lin[5] / l;
  c->hlin[6] = c->lin[6] / (cp * l * l);
  c->hlin[7] = c->lin[7] / (cp * l);
  c->hlin[8] = c->lin[8] / (l * l);
  return LBM_OK;
}

}  // namespace lbm

// ----------------------------------------------------------- kernels ----

namespace {

// nodes per block of the one-step kernel: 15 wavefronts and one more for the
// halo (960 against 256 nodes per block: 60.7 -> 61.4 GLUPS at N = 2^24)
constexpr int kPlainBlock = 960;
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

// One time step, one node per thread.  Block b stores nodes
// [b*B, b*B + B) (B = kPlainBlock), each thread its own node with aligned
// stores: the streamed values f+(j) = f+*(j-1) and f-(j) = f-*(j+1) come
// through LDS.  One more wavefront handles the four halo nodes: b*B - 1 and
// b*B + B are collided too (their f+* and f-* stream into the block), and
// b*B - 2, b*B + B + 1 give u, T for those two nodes' sources.  LDS slot s
// holds node b*B - 2 + s.  NT: non-temporal loads and stores, for states far
// larger than the caches (measured on a 6-array copy: 6.1 against 5.6 TB/s;
// with stores shifted by one node, as push streaming writes them, 5.5).
template <int EQ, bool NT>
__global__ __launch_bounds__(kPlainBlock + 64) void k_step_plain(
    Consts c, const double* __restrict__ fin, double* __restrict__ fout,
    int64_t n) {
  constexpr int NS = kPlainBlock + 4;
  __shared__ double su[NS], sT[NS], sfp[NS], sgp[NS], sfm[NS], sgm[NS];
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * kPlainBlock;
  const int64_t rem = n - b0;
  const int nloc = rem < kPlainBlock ? (int)rem : kPlainBlock;
  // this thread's node and LDS slot; -1: no node
  int slot = -1;
  int64_t j = 0;
  if (tid < kPlainBlock) {
    if (tid < nloc) {
      slot = tid + 2;
      j = b0 + tid;
    }
  } else if (tid < kPlainBlock + 4) {
    const int h = tid - kPlainBlock;  // b0-2, b0-1, b0+nloc, b0+nloc+1
    slot = h < 2 ? h : nloc + h;
    j = lbm::wrap_mod(b0 - 2 + slot, n);
  }
  const bool own = tid < nloc;
  const bool collide = slot >= 1 && slot <= nloc + 2;
  double f0 = 0, fp = 0, fm = 0, g0 = 0, gp = 0, gm = 0, u = 0, T = 0, rw = 0,
         w = 0;
  if (slot >= 0) {
    if (NT) {
      f0 = __builtin_nontemporal_load(&fin[j]);
      fp = __builtin_nontemporal_load(&fin[n + j]);
      fm = __builtin_nontemporal_load(&fin[2 * n + j]);
      g0 = __builtin_nontemporal_load(&fin[3 * n + j]);
      gp = __builtin_nontemporal_load(&fin[4 * n + j]);
      gm = __builtin_nontemporal_load(&fin[5 * n + j]);
    } else {
      f0 = fin[j];
      fp = fin[n + j];
      fm = fin[2 * n + j];
      g0 = fin[3 * n + j];
      gp = fin[4 * n + j];
      gm = fin[5 * n + j];
    }
    if (collide)
      lbm::collide_local<EQ>(c, f0, fp, fm, g0, gp, gm, u, T, rw, w);
    else
      lbm::node_uT(c, f0, fp, fm, g0, gp, gm, u, T);
    su[slot] = u;
    sT[slot] = T;
  }
  __syncthreads();
  if (collide) {
    const double add = lbm::source_g(c, rw, w, su[slot - 1], su[slot + 1],
                                     sT[slot - 1], sT[slot + 1]);
    g0 += add;
    gp += add;
    gm += add;
    sfp[slot] = fp;
    sgp[slot] = gp;
    sfm[slot] = fm;
    sgm[slot] = gm;
  }
  __syncthreads();
  if (!own) return;
  // (viii) streaming, pulled from the neighbours' post-collision values
  fp = sfp[slot - 1];
  gp = sgp[slot - 1];
  fm = sfm[slot + 1];
  gm = sgm[slot + 1];
  if (NT) {
    __builtin_nontemporal_store(f0, &fout[j]);
    __builtin_nontemporal_store(fp, &fout[n + j]);
    __builtin_nontemporal_store(fm, &fout[2 * n + j]);
    __builtin_nontemporal_store(g0, &fout[3 * n + j]);
    __builtin_nontemporal_store(gp, &fout[4 * n + j]);
    __builtin_nontemporal_store(gm, &fout[5 * n + j]);
  } else {
    fout[j] = f0;
    fout[n + j] = fp;
    fout[2 * n + j] = fm;
    fout[3 * n + j] = g0;
    fout[4 * n + j] = gp;
    fout[5 * n + j] = gm;
  }
}

// K time steps of one register-resident tile per workgroup (see the file
// header).  The workgroup has WG wavefronts of 64 lanes, lane l of wavefront
// w holding the P consecutive nodes starting at tile index w*62P + (l-1)P
// (l = 0..63; wavefront 0 starts at tile index 0).  Neighbouring wavefronts
// overlap by two lanes: lane 0 of wavefront w > 0 mirrors lane 62 of w-1,
// lane 63 of w < WG-1 mirrors lane 1 of w+1.  A tile thus spans
// tile_nodes = P(62 WG + 2) nodes; tile t stores nodes [t*OUT, t*OUT + OUT)
// with OUT = tile_nodes - 4K and loads [t*OUT - 2K, t*OUT + OUT + 2K)
// (periodic).
//
// Every step runs within the wavefront (lane neighbours through DPP).  The
// outermost lanes have no neighbour there; as one step has radius 2, the
// error this leaves at a mirror lane's outer end moves two nodes inwards per
// step and reaches the wavefront's own lanes after P/2 steps.  So every P/2
// steps the wavefronts copy their edge lanes 1 and 62 into the neighbours'
// mirror lanes through LDS (one workgroup barrier per copy, double-buffered);
// each wavefront stores only its own lanes.  The error at the tile's two
// outer ends is what the halo of 2K nodes absorbs.
//
// Refresh of the mirror lanes: lanes 1 and 62 publish their populations in
// `edge` (one buffer of the double-buffered pair: a buffer is written again
// only after the next refresh's barrier, which every reader of its previous
// contents has passed), then lane 0 takes lane 62 of the wavefront to its
// left and lane 63 lane 1 of the wavefront to its right.
template <int P, int WG>
__device__ __forceinline__ void mirror_refresh(double (&f)[6][P],
                                               double (*edge)[2][6 * P],
                                               int lane, int wave, int nw) {
  if (lane == 1 || lane == 62) {
    double* d = edge[wave][lane == 62];
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) d[q * P + k] = f[q][k];
  }
  __syncthreads();
  const bool left = lane == 0 && wave > 0, right = lane == 63 && wave < nw - 1;
  if (left || right) {
    const double* e = left ? edge[wave - 1][1] : edge[wave + 1][0];
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) f[q][k] = e[q * P + k];
  }
}

// Active wavefronts of a tile that starts at lattice index `start` (halo H)
// in a lattice of n nodes: the fewest of the WG whose span P(62 nw + 2)
// still covers the nodes the tile stores plus both halos.  Only a lattice's
// last tile, or a lattice shorter than one tile, needs fewer than WG.
template <int P, int WG>
__device__ __forceinline__ int active_waves(int64_t n, int64_t start, int H) {
  const int64_t store = n - (start + H);  // nodes from the tile's first output
  const int64_t need = store + 2 * H - 2 * P;  // span - 2P the tile needs
  if (need >= (int64_t)62 * P * WG) return WG;
  const int nw = (int)((need + 62 * P - 1) / (62 * P));
  return nw < 1 ? 1 : nw;
}

// Tile t of a lattice of n nodes (array stride S) starting at lattice index
// `start` = t*OUT - H, OUT = tile_nodes - 2H: load, K <= H/2 steps, store of
// the interior [H, span - H) (one step has radius 2, so K steps need
// H >= 2K).  Only the first nw wavefronts work (span P(62 nw + 2)); the
// others end at once, which a workgroup barrier allows (it waits for the
// wavefronts that have not ended), and leave their SIMDs to other
// workgroups.  With every_step (the recompute of a checkpoint segment for a
// reverse sweep), the state after step s = 1..K is state i = first + s of
// the segment, and the interior of those states whose i is a multiple of
// `every` is stored, state i into fout + ((i-1)/every)*state_stride.
template <int P, int WG, int EQ>
__device__ __forceinline__ void tile_run(const Consts& c,
                                         const double* __restrict__ fin,
                                         double* __restrict__ fout, int64_t S,
                                         int64_t n, int64_t start, int H,
                                         int K, bool every_step = false,
                                         int64_t state_stride = 0,
                                         int first = 0, int every = 1) {
  // one node per lane leaves no room for mirror lanes: one wavefront
  static_assert(P > 1 || WG == 1, "P = 1 tiles have one wavefront");
  constexpr int WW = 64 * P;       // nodes of one wavefront
  constexpr int WS = 62 * P;       // wavefront stride in the tile
  __shared__ double stage[WG * (WW + 64)];
  __shared__ double edge[2][WG][2][6 * P];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = active_waves<P, WG>(n, start, H);
  if (wave >= nw) return;  // uniform over the wavefront
  const int W = lbm::tile_nodes(P, nw);
  double* lds = stage + wave * (WW + 64);
  const int64_t wstart = start + wave * WS;
  const bool inside = start >= 0 && start + W <= n;
  const bool small = n < W;
  double f[6][P];
  tile_load<P>(fin, S, n, wstart, inside, small, lane, lds, f);
  // the tile's valid indices [H, W - H), in this wavefront's numbering and
  // restricted to its own lanes (the mirror lanes belong to the neighbours)
  const int lo = max(H - wave * WS, wave > 0 ? P : 0);
  const int hi = min(W - H - wave * WS, wave < nw - 1 ? WW - P : WW);
  int since = 0, buf = 0;
  for (int step = 0; step < K; ++step) {
    tile_step<P, EQ>(c, f);
    if (every_step && (first + step + 1) % every == 0)
      tile_store<P>(fout + (int64_t)((first + step) / every) * state_stride, S,
                    n, wstart, lo, hi, lane, lds, f);
    if (WG > 1 && ++since == P / 2 && step + 1 < K) {
      mirror_refresh<P, WG>(f, edge[buf], lane, wave, nw);
      buf ^= 1;
      since = 0;
    }
  }
  if (!every_step) tile_store<P>(fout, S, n, wstart, lo, hi, lane, lds, f);
}

// Wavefronts per SIMD the tile kernels are compiled for (the register
// budget: 512 / n VGPRs each).  Section-8 kernels at P = 8 hold 168 VGPRs
// for three (the few values that spill are touched only around the step
// loop, which measured 297 -> 312 GLUPS at N = 2^24 against two); with 8
// wavefronts per workgroup a CU gains no third one, so those stay at two.
// The kernels that select the equilibria per lattice, or store the states
// of a reverse sweep, need more registers at P >= 4 and take one.  P <= 2
// needs few registers: four.
constexpr int tile_waves_per_simd(int P, int WG, bool sec8_plain) {
  return P <= 2 ? 4 : (!sec8_plain ? 1 : (P == 8 && WG <= 4 ? 3 : 2));
}

template <int P, int WG, int EQ>
__global__ __launch_bounds__(64 * WG, tile_waves_per_simd(P, WG, EQ == 0)) void k_step_tile(
    Consts c, const double* __restrict__ fin, double* __restrict__ fout,
    int64_t n, int K, int64_t ntiles) {
  const int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;  // uniform over the workgroup
  const int OUT = lbm::tile_nodes(P, WG) - 4 * K;
  tile_run<P, WG, EQ>(c, fin, fout, n, n, tile * OUT - 2 * K, 2 * K, K);
}

// Batched form: workgroup b advances tile tiles[b].t of lattice tiles[b].inst,
// which occupies [offs[inst], offs[inst+1]) of every array of a state of
// array stride S, with that lattice's own constants.  The tiling (halo H,
// OUT = W - 2H) is fixed by the tile table; a launch runs K <= H/2 steps.
// EVERY: store the states of a checkpoint segment that the reverse sweep
// loads (see tile_run: first, every).
template <int P, int WG, int EQ, bool EVERY>
__global__ __launch_bounds__(64 * WG, tile_waves_per_simd(P, WG, EQ == 0 && !EVERY)) void k_batch_tile(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const lbm::TileRef* __restrict__ tiles, const double* __restrict__ fin,
    double* __restrict__ fout, int64_t S, int H, int K, int64_t ntiles,
    int64_t state_stride, int first, int every) {
  const int64_t b = blockIdx.x;
  if (b >= ntiles) return;  // uniform over the workgroup
  const lbm::TileRef tr = tiles[b];
  const int64_t off = offs[tr.inst];
  const int64_t n = offs[tr.inst + 1] - off;
  const Consts c = cs[tr.inst];
  const int OUT = lbm::tile_nodes(P, WG) - 2 * H;
  tile_run<P, WG, EQ>(c, fin + off, fout + off, S, n, (int64_t)tr.t * OUT - H, H,
                  K, EVERY, state_stride, first, every);
}

// Resident lattices of a batch: a periodic lattice of L nodes short enough
// for the registers of one workgroup runs every time step of the call in one
// launch, with no halo and no global memory traffic between the first load
// and the last store.  The lattice is laid out as a tile that starts at
// position -P: lane l of its wavefront w (w = 0 .. nw-1, nw = ceil(L / 62P))
// holds positions 62 P w + P (l - 1) + k, neighbouring wavefronts sharing
// two lanes as in the tile kernels.  Positions outside [0, L) stand for the
// nodes their periodic image names: lane 0 of wavefront 0 holds nodes
// L-P .. L-1 and positions L .. L+P-1 hold nodes 0 .. P-1; every P/2 steps
// those copies and the mirror lanes are refreshed from the lanes that own
// the nodes, through LDS with one workgroup barrier (every lattice of a
// workgroup runs the same steps, so all its wavefronts meet at each).  A
// step has radius 2, so the wrong values that come in from beyond a copy
// (or from the unused positions past L+P) move two nodes per step and stay
// inside the copy until the refresh, as for the mirror lanes.  Several
// lattices share a workgroup of kResWaves wavefronts (items[wg_first[b] ..
// wg_first[b+1]), each on its own wavefronts); wavefronts without a
// lattice end at once.
// Every node-update rounds as in the other kernels: results are bitwise
// those of the tiled path.
constexpr int kResWaves = lbm::kResidentWaves;

// The copies of the periodic wrap, in P-node blocks: every lane holds the
// P positions p0 .. p0+P-1 with p0 a multiple of P, so with o = L mod P
// the nodes L-P .. L-1 are the last P - o nodes of the owner lane at
// L-P-o followed by the first o of the owner lane at L-o, and the
// positions L .. L+P-1 are the last P - o of the lane at L-o (every lane
// holding that block: a mirror lane as well) followed by the first o of
// the lane at L-o+P.  Those owners write their whole P nodes into a 2P-node
// buffer read at offset o, which keeps the exchange free of per-node
// conditions.
template <int P>
__device__ __forceinline__ void resident_refresh(
    double (&f)[6][P], double (*edge)[2][6 * P], double (*head)[6 * P],
    double (*tail)[12 * P], int lane, int wave, int lw, int nw, int w0,
    int L) {
  const int p0 = 62 * P * lw + P * (lane - 1);  // position of node 0 of the lane
  const int o = L % P;                          // uniform over the lattice
  if (lane == 1 || lane == 62) {
    double* d = edge[wave][lane == 62];
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) d[q * P + k] = f[q][k];
  }
  if (lw == 0 && lane == 1) {  // nodes 0 .. P-1
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) head[w0][q * P + k] = f[q][k];
  }
  const bool owner = lane >= 1 && lane <= 62;
  if (owner && (p0 == L - P - o || (o != 0 && p0 == L - o))) {  // nodes L-P .. L-1
    double* d = tail[w0] + (p0 == L - o ? P : 0);
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) d[q * 2 * P + k] = f[q][k];
  }
  __syncthreads();
  if (lane == 0 && lw > 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) f[q][k] = edge[wave - 1][1][q * P + k];
  } else if (lane == 63 && lw < nw - 1) {
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) f[q][k] = edge[wave + 1][0][q * P + k];
  } else if (lane == 0) {  // lw == 0: nodes L-P .. L-1
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) f[q][k] = tail[w0][q * 2 * P + o + k];
  }
  // positions L .. L+P-1 (nodes 0 .. P-1 again), after the mirror reads
  if (p0 == L - o) {
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k)
        if (k >= o) f[q][k] = head[w0][q * P + k - o];
  } else if (o != 0 && p0 == L - o + P) {
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k)
        if (k < o) f[q][k] = head[w0][q * P + P - o + k];
  }
}

template <int P, int EQ>
__global__ __launch_bounds__(64 * kResWaves, 3) void k_batch_resident(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const lbm::ResidentItem* __restrict__ items,
    const int32_t* __restrict__ wg_first, const double* fin, double* fout,
    int64_t S, int64_t T) {
  // fin and fout may be the same state (the run is in place): no restrict
  constexpr int WG = kResWaves;
  constexpr int WW = 64 * P;
  constexpr int WS = 62 * P;
  __shared__ double stage[WG * (WW + 64)];
  __shared__ double edge[2][WG][2][6 * P];
  __shared__ double head[2][WG][6 * P];
  __shared__ double tail[2][WG][12 * P];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // this wavefront's lattice (uniform over the wavefront)
  int item = -1;
  for (int i = wg_first[blockIdx.x]; i < wg_first[blockIdx.x + 1]; ++i) {
    const int w0 = items[i].wave0;
    if (wave >= w0 && wave < w0 + items[i].nw) item = i;
  }
  if (item < 0) return;
  const lbm::ResidentItem it = items[item];
  const int lw = wave - it.wave0;
  const int64_t off = offs[it.inst];
  const int L = (int)(offs[it.inst + 1] - off);
  const Consts c = cs[it.inst];
  double* lds = stage + wave * (WW + 64);
  const int64_t wstart = -P + (int64_t)lw * WS;
  double f[6][P];
  tile_load<P>(fin + off, S, L, wstart, false, true, lane, lds, f);
  // every wavefront has loaded before any stores (fout may be fin)
  __syncthreads();
  int since = 0, buf = 0;
  for (int64_t step = 0; step < T; ++step) {
    tile_step<P, EQ>(c, f);
    if (++since == P / 2 && step + 1 < T) {
      resident_refresh<P>(f, edge[buf], head[buf], tail[buf], lane, wave, lw,
                          it.nw, it.wave0, L);
      buf ^= 1;
      since = 0;
    }
  }
  // owned positions 0 .. L-1: lanes 1 .. 62, and 63 in the last wavefront
  tile_store<P>(fout + off, S, L, wstart, P, lw < it.nw - 1 ? WW - P : WW, lane,
                lds, f);
}

// One workgroup per lattice of a batch: moments m = M f (eq. M-d1q3q3).
__global__ __launch_bounds__(256) void k_batch_moments(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const double* __restrict__ f, double* __restrict__ m, int64_t S) {
  const int inst = blockIdx.x;
  const Consts c = cs[inst];
  for (int64_t j = offs[inst] + threadIdx.x; j < offs[inst + 1]; j += 256) {
    const double f0 = f[j], fp = f[S + j], fm = f[2 * S + j];
    const double g0 = f[3 * S + j], gp = f[4 * S + j], gm = f[5 * S + j];
    const double sf = fp + fm, sg = gp + gm;
    m[j] = lbm::density(c, f0, fp, fm);
    m[S + j] = c.mJ * (fp - fm);
    m[2 * S + j] = c.mz * (g0 + sg);
    m[3 * S + j] = c.me * (sf - 2.0 * f0);
    m[4 * S + j] = c.mpsi * (gp - gm);
    m[5 * S + j] = c.meps * (sg - 2.0 * g0);
  }
}

// One workgroup per lattice of a batch: equilibrium populations.
__global__ __launch_bounds__(256) void k_batch_equilibrium(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const double* __restrict__ rho, const double* __restrict__ J,
    const double* __restrict__ zeta, double* __restrict__ f, int64_t S) {
  const int inst = blockIdx.x;
  const Consts c = cs[inst];
  for (int64_t j = offs[inst] + threadIdx.x; j < offs[inst + 1]; j += 256) {
    double v[6];
    lbm::equilibrium(c, rho[j], J[j], zeta[j], v);
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k * S + j] = v[k];
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

// Per-lattice diagnostics of a batch, one workgroup per lattice, fixed tree
// order; out[8*inst + k] as in lbm_diagnostics.
__global__ __launch_bounds__(kDiagBlock) void k_batch_diag(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const double* __restrict__ f, int64_t S, double* __restrict__ out) {
  __shared__ double s[kDiagBlock][8];
  const int inst = blockIdx.x;
  const Consts c = cs[inst];
  double a[8] = {0, 0, 0, 0, INFINITY, INFINITY, 0, 0};
  for (int64_t j = offs[inst] + threadIdx.x; j < offs[inst + 1];
       j += kDiagBlock) {
    const double f0 = f[j], fp = f[S + j], fm = f[2 * S + j];
    const double g0 = f[3 * S + j], gp = f[4 * S + j], gm = f[5 * S + j];
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
  if (threadIdx.x < 8) out[8 * inst + threadIdx.x] = s[0][threadIdx.x];
}

// ------------------------------------------------- failure detection ---
//
// LBM_CHECK_FINITE: after a launch, every node the launch wrote is checked
// as lbm_diagnostics counts it: its six populations finite, rho > 0 and
// T > 0 (T from the equation of state).  A failing node gives the key
// (steps << shift) | index, with steps the time steps done when the launch
// ended and index its node (single lattice) or lattice (batch); the record
// keeps the smallest key: each lane's minimum over its nodes, the wavefront's
// minimum by a butterfly, then one 64-bit vector atomic min per wavefront.

__device__ __forceinline__ bool node_fails(const Consts& c,
                                           const double* __restrict__ f,
                                           int64_t S, int64_t j) {
  const double f0 = f[j], fp = f[S + j], fm = f[2 * S + j];
  const double g0 = f[3 * S + j], gp = f[4 * S + j], gm = f[5 * S + j];
  const bool finite = isfinite(f0) && isfinite(fp) && isfinite(fm) &&
                      isfinite(g0) && isfinite(gp) && isfinite(gm);
  const double rho = lbm::density(c, f0, fp, fm);
  const double J = c.mJ * (fp - fm);
  const double zeta = c.mz * (g0 + (gp + gm));
  double u, s_, X, T;
  lbm::thermo(c, rho, J, zeta, u, s_, X, T);
  return !(finite && rho > 0.0 && T > 0.0);
}

// Every lane of the wavefront takes part (lanes without a failing node
// bring ~0).
__device__ __forceinline__ void record_min(unsigned long long* rec,
                                           unsigned long long key) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const unsigned long long o = __shfl_xor(key, m, 64);
    key = o < key ? o : key;
  }
  if ((threadIdx.x & 63) == 0 && key != ~0ull) atomicMin(rec, key);
}

__global__ __launch_bounds__(64) void k_check_reset(unsigned long long* rec) {
  if (threadIdx.x == 0) *rec = ~0ull;
}

// Single lattice: nodes [0, n), key steps_key | j.
__global__ __launch_bounds__(256) void k_check_state(
    Consts c, const double* __restrict__ f, int64_t n,
    unsigned long long steps_key, unsigned long long* rec) {
  unsigned long long key = ~0ull;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * 256)
    if (node_fails(c, f, n, j) && (steps_key | (unsigned long long)j) < key)
      key = steps_key | (unsigned long long)j;
  record_min(rec, key);
}

// Batch: workgroup b checks the nodes tile tiles[b] stored, [t OUT,
// t OUT + OUT) of its lattice, if that lattice asks for it; key
// steps_key | inst.
__global__ __launch_bounds__(256) void k_batch_check(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const lbm::TileRef* __restrict__ tiles, const double* __restrict__ f,
    int64_t S, int OUT, unsigned long long steps_key,
    unsigned long long* rec) {
  const lbm::TileRef tr = tiles[blockIdx.x];
  if (!(cs[tr.inst].flags & LBM_CHECK_FINITE)) return;  // uniform
  const Consts c = cs[tr.inst];
  const int64_t off = offs[tr.inst];
  const int64_t n = offs[tr.inst + 1] - off;
  const int64_t lo = (int64_t)tr.t * OUT;
  const int64_t hi = lo + OUT < n ? lo + OUT : n;
  bool bad = false;
  for (int64_t j = lo + threadIdx.x; j < hi; j += 256)
    bad = bad || node_fails(c, f + off, S, j);
  record_min(rec, bad ? steps_key | (unsigned long long)tr.inst : ~0ull);
}

// Checks (LBM_CHECK_FINITE) of the resident lattices, one workgroup per
// item, those whose flags ask for it; key steps_key | inst.
__global__ __launch_bounds__(256) void k_batch_check_lattices(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const lbm::ResidentItem* __restrict__ items, const double* __restrict__ f,
    int64_t S, unsigned long long steps_key, unsigned long long* rec) {
  const int inst = items[blockIdx.x].inst;
  if (!(cs[inst].flags & LBM_CHECK_FINITE)) return;  // uniform
  const Consts c = cs[inst];
  const int64_t off = offs[inst];
  const int64_t n = offs[inst + 1] - off;
  bool bad = false;
  for (int64_t j = threadIdx.x; j < n; j += 256) bad = bad || node_fails(c, f + off, S, j);
  record_min(rec, bad ? steps_key | (unsigned long long)inst : ~0ull);
}

// Copy of the nodes [t OUT, t OUT + OUT) of tile b's lattice from src to
// dst, one workgroup per tile: brings back into the caller's state the
// lattices of a launch sequence that ended in the workspace state.
__global__ __launch_bounds__(256) void k_batch_copy_tiles(
    const int64_t* __restrict__ offs, const lbm::TileRef* __restrict__ tiles,
    int OUT, const double* __restrict__ src, double* __restrict__ dst,
    int64_t S) {
  const lbm::TileRef tr = tiles[blockIdx.x];
  const int64_t off = offs[tr.inst];
  const int64_t n = offs[tr.inst + 1] - off;
  const int64_t lo = off + (int64_t)tr.t * OUT;
  const int64_t hi = off + ((int64_t)tr.t * OUT + OUT < n ? (int64_t)tr.t * OUT + OUT : n);
  for (int64_t j = lo + threadIdx.x; j < hi; j += 256)
#pragma unroll
    for (int q = 0; q < 6; ++q) dst[q * S + j] = src[q * S + j];
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
  const dim3 grid((unsigned)cdiv(n, kPlainBlock)), block(kPlainBlock + 64);
  // non-temporal accesses once the two states (96 B per node) outgrow the
  // 256 MB of on-die cache
  const bool nt = 96 * n > (int64_t(256) << 20);
  if (c.eq_kind == 0 && nt)
    hipLaunchKernelGGL((k_step_plain<0, true>), grid, block, 0, s, c, fin, fout, n);
  else if (c.eq_kind == 0)
    hipLaunchKernelGGL((k_step_plain<0, false>), grid, block, 0, s, c, fin, fout, n);
  else if (nt)
    hipLaunchKernelGGL((k_step_plain<-1, true>), grid, block, 0, s, c, fin, fout, n);
  else
    hipLaunchKernelGGL((k_step_plain<-1, false>), grid, block, 0, s, c, fin, fout, n);
  return hip_check(hipGetLastError(), "k_step_plain");
}

int64_t tile_out(int P, int K, int wg) { return tile_nodes(P, wg) - 4 * K; }

template <int P, int WG>
static void launch_tile_t(const Consts& c, const double* fin, double* fout,
                          int64_t n, int K, hipStream_t s) {
  const int64_t ntiles = cdiv(n, tile_out(P, K, WG));
  if (c.eq_kind == 0)
    hipLaunchKernelGGL((k_step_tile<P, WG, 0>), dim3((unsigned)ntiles),
                       dim3(64 * WG), 0, s, c, fin, fout, n, K, ntiles);
  else
    hipLaunchKernelGGL((k_step_tile<P, WG, -1>), dim3((unsigned)ntiles),
                       dim3(64 * WG), 0, s, c, fin, fout, n, K, ntiles);
}

template <int P>
static int launch_tile_p(const Consts& c, const double* fin, double* fout,
                         int64_t n, int K, int wg, hipStream_t s) {
  switch (wg) {
    case 1: launch_tile_t<P, 1>(c, fin, fout, n, K, s); break;
    case 2: launch_tile_t<P, 2>(c, fin, fout, n, K, s); break;
    case 4: launch_tile_t<P, 4>(c, fin, fout, n, K, s); break;
    case 8: launch_tile_t<P, 8>(c, fin, fout, n, K, s); break;
    default: return set_err(LBM_EINVAL, "waves_per_group must be 1, 2, 4 or 8");
  }
  return LBM_OK;
}

int launch_step_tile(const Consts& c, const double* fin, double* fout,
                     int64_t n, int P, int K, int wpg, hipStream_t s) {
  int rc;
  switch (P) {
    case 1:
      if (wpg != 1) return set_err(LBM_EINVAL, "nodes_per_lane 1 needs one wavefront");
      launch_tile_t<1, 1>(c, fin, fout, n, K, s);
      rc = LBM_OK;
      break;
    case 2: rc = launch_tile_p<2>(c, fin, fout, n, K, wpg, s); break;
    case 4: rc = launch_tile_p<4>(c, fin, fout, n, K, wpg, s); break;
    case 8: rc = launch_tile_p<8>(c, fin, fout, n, K, wpg, s); break;
    default: return set_err(LBM_EINVAL, "nodes_per_lane must be 1, 2, 4 or 8");
  }
  if (rc) return rc;
  return hip_check(hipGetLastError(), "k_step_tile");
}

// reduction scratch of the diagnostics (8 final values, 8 per block), then
// the failure record of LBM_CHECK_FINITE (4 doubles)
size_t diag_ws_doubles() { return (size_t)kDiagMaxBlocks * 8 + 8 + 4; }
size_t check_record_double() { return (size_t)kDiagMaxBlocks * 8 + 8; }

int launch_check_reset(unsigned long long* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_check_reset, dim3(1), dim3(64), 0, s, rec);
  return hip_check(hipGetLastError(), "k_check_reset");
}

int launch_check_state(const Consts& c, const double* f, int64_t n,
                       int64_t steps, unsigned long long* rec, hipStream_t s) {
  const unsigned long long sk =
      (unsigned long long)std::min<int64_t>(steps, kCheckMaxSteps1) << 36;
  const int nb = (int)std::min<int64_t>(2048, cdiv(n, 256));
  hipLaunchKernelGGL(k_check_state, dim3(nb), dim3(256), 0, s, c, f, n, sk, rec);
  return hip_check(hipGetLastError(), "k_check_state");
}

int launch_batch_check(const Consts* cs, const int64_t* offs,
                       const TileRef* tiles, int64_t ntiles, const double* f,
                       int64_t S, int OUT, int64_t steps,
                       unsigned long long* rec, hipStream_t s) {
  if (ntiles <= 0) return LBM_OK;
  const unsigned long long sk =
      (unsigned long long)std::min<int64_t>(steps, kCheckMaxStepsB) << 31;
  hipLaunchKernelGGL(k_batch_check, dim3((unsigned)ntiles), dim3(256), 0, s, cs,
                     offs, tiles, f, S, OUT, sk, rec);
  return hip_check(hipGetLastError(), "k_batch_check");
}

int launch_batch_copy_tiles(const int64_t* offs, const TileRef* tiles,
                            int64_t ntiles, int OUT, const double* src,
                            double* dst, int64_t S, hipStream_t s) {
  if (ntiles <= 0) return LBM_OK;
  hipLaunchKernelGGL(k_batch_copy_tiles, dim3((unsigned)ntiles), dim3(256), 0, s,
                     offs, tiles, OUT, src, dst, S);
  return hip_check(hipGetLastError(), "k_batch_copy_tiles");
}

int launch_batch_resident(const Consts* cs, const int64_t* offs,
                          const ResidentItem* items, const int32_t* wg_first,
                          int64_t nwg, const double* fin, double* fout,
                          int64_t S, int64_t T, int eq, hipStream_t s) {
  if (nwg <= 0 || T <= 0) return LBM_OK;
  if (eq != 0)
    return set_err(LBM_EINVAL, "resident lattices need the section-8 equilibria");
  hipLaunchKernelGGL((k_batch_resident<kResP, 0>), dim3((unsigned)nwg),
                     dim3(64 * kResWaves), 0, s, cs, offs, items, wg_first, fin,
                     fout, S, T);
  return hip_check(hipGetLastError(), "k_batch_resident");
}

int launch_batch_check_lattices(const Consts* cs, const int64_t* offs,
                                const ResidentItem* items, int64_t nitems,
                                const double* f, int64_t S, int64_t steps,
                                unsigned long long* rec, hipStream_t s) {
  if (nitems <= 0) return LBM_OK;
  const unsigned long long sk =
      (unsigned long long)std::min<int64_t>(steps, kCheckMaxStepsB) << 31;
  hipLaunchKernelGGL(k_batch_check_lattices, dim3((unsigned)nitems), dim3(256), 0,
                     s, cs, offs, items, f, S, sk, rec);
  return hip_check(hipGetLastError(), "k_batch_check_lattices");
}

int read_check_record(const unsigned long long* rec, hipStream_t s,
                      unsigned long long* out) {
  int rc = hip_check(hipMemcpyAsync(out, rec, sizeof *out, hipMemcpyDeviceToHost, s),
                     "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  return rc;
}

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

template <int P, int WG>
static void launch_batch_t(const Consts* cs, const int64_t* offs,
                           const TileRef* tiles, int64_t ntiles,
                           const double* fin, double* fout, int64_t S, int H,
                           int K, int64_t state_stride, int first, int every,
                           int eq, hipStream_t s) {
  const dim3 grid((unsigned)ntiles), block(64 * WG);
  if (eq == 0 && state_stride == 0)
    hipLaunchKernelGGL((k_batch_tile<P, WG, 0, false>), grid, block, 0, s, cs,
                       offs, tiles, fin, fout, S, H, K, ntiles, state_stride, first,
                       every);
  else if (eq == 0)
    hipLaunchKernelGGL((k_batch_tile<P, WG, 0, true>), grid, block, 0, s, cs,
                       offs, tiles, fin, fout, S, H, K, ntiles, state_stride, first,
                       every);
  else if (state_stride == 0)
    hipLaunchKernelGGL((k_batch_tile<P, WG, -1, false>), grid, block, 0, s, cs,
                       offs, tiles, fin, fout, S, H, K, ntiles, state_stride, first,
                       every);
  else
    hipLaunchKernelGGL((k_batch_tile<P, WG, -1, true>), grid, block, 0, s, cs,
                       offs, tiles, fin, fout, S, H, K, ntiles, state_stride, first,
                       every);
}

int launch_batch_tile(const Consts* cs, const int64_t* offs,
                      const TileRef* tiles, int64_t ntiles, const double* fin,
                      double* fout, int64_t S, int P, int H, int K, int wg,
                      int eq, hipStream_t s, int64_t state_stride, int first,
                      int every) {
  if (ntiles <= 0) return LBM_OK;
  if (K < 1 || 2 * K > H || 2 * H >= tile_nodes(P, wg))
    return set_err(LBM_EINVAL, "bad batched tile geometry H=%d K=%d", H, K);
  if (first < 0 || every < 1)
    return set_err(LBM_EINVAL, "bad segment state numbering");
#define LBM_BATCH_CASE(PP, WW)                                              \
  if (P == PP && wg == WW) {                                                \
    launch_batch_t<PP, WW>(cs, offs, tiles, ntiles, fin, fout, S, H, K,    \
                           state_stride, first, every, eq, s);              \
    return hip_check(hipGetLastError(), "k_batch_tile");                    \
  }
  LBM_BATCH_CASE(1, 1)
  LBM_BATCH_CASE(2, 1)
  LBM_BATCH_CASE(2, 2)
  LBM_BATCH_CASE(2, 4)
  LBM_BATCH_CASE(2, 8)
  LBM_BATCH_CASE(4, 1)
  LBM_BATCH_CASE(4, 2)
  LBM_BATCH_CASE(4, 4)
  LBM_BATCH_CASE(4, 8)
  LBM_BATCH_CASE(8, 1)
  LBM_BATCH_CASE(8, 2)
  LBM_BATCH_CASE(8, 4)
  LBM_BATCH_CASE(8, 8)
#undef LBM_BATCH_CASE
  return set_err(LBM_EINVAL, "unsupported tile shape P=%d waves=%d", P, wg);
}

int launch_batch_equilibrium(const Consts* cs, const int64_t* offs,
                             int64_t n_inst, const double* rho, const double* J,
                             const double* zeta, double* f, int64_t S,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_batch_equilibrium, dim3((unsigned)n_inst), dim3(256), 0,
                     s, cs, offs, rho, J, zeta, f, S);
  return hip_check(hipGetLastError(), "k_batch_equilibrium");
}

int launch_batch_moments(const Consts* cs, const int64_t* offs, int64_t n_inst,
                         const double* f, double* m, int64_t S, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_moments, dim3((unsigned)n_inst), dim3(256), 0, s,
                     cs, offs, f, m, S);
  return hip_check(hipGetLastError(), "k_batch_moments");
}

int launch_batch_diag(const Consts* cs, const int64_t* offs, int64_t n_inst,
                      const double* f, int64_t S, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_diag, dim3((unsigned)n_inst), dim3(kDiagBlock), 0,
                     s, cs, offs, f, S, out);
  return hip_check(hipGetLastError(), "k_batch_diag");
}

}  // namespace lbm
