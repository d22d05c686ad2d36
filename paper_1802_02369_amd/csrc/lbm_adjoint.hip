// Reverse mode of the coupled D1Q3Q3 time step (Dubois, Graille & Lallemand,
// arXiv 1802.02369, section 8, steps (i)-(viii)): adjoint kernels, loss and
// seed, checkpointed forward and reverse drivers, for batches of lattices (a
// single lattice is a batch of one).  Declared in include/lbm.h.
//
// Adjoint of one step, node j, given fbar(t+1) (the gradient with respect to
// the state after the step):
//   (viii)^T  fbar*_0(j) = fbar_0(t+1, j), fbar*_+(j) = fbar_+(t+1, j+1),
//             fbar*_-(j) = fbar_-(t+1, j-1) (same for g);
//   (vi)^T    adjoints of (rho, J, zeta + dz, e*, psi*, eps*) = M^-T fbar*;
//   (vii)^T   dz_i = c rho_i w_i [du_i^2 + (cp/Pr) dT_i^2 w_i], w = 1/T,
//             du_i = u_{i+1} - u_{i-1}, dT_i = T_{i+1} - T_{i-1},
//             c = (1/s_e - 1/2)/4, depends on u, T of i-1 and i+1: node j
//             gathers 2 c rho w du zbar and 2 c (cp/Pr) rho w^2 dT zbar from
//             its two neighbours (the transposed scatter of the forward);
//   (v)^T, (iv)^T, (ii)^T  the local chain through the relaxation, the
//             equilibria and the equation of state back to f(t, j);
//   rates     d/ds_e (relaxation of e and c), d/ds_psi, d/ds_eps.
// The step has radius 2 in both f(t) and fbar(t+1).  Two kernels run it:
// k_adjoint_step, one step per launch, one thread per node, 256-node tiles
// whose 252 interior nodes are stored, u, T and the gathered terms through
// LDS; and k_adjoint_tile, up to K steps per launch on a register tile (the
// default where its tiles hold the halo; see below), which on large problems
// loads every second forward state and recomputes the others.  The sweep
// recomputes each checkpoint segment's states before its reverse steps
// (enqueue_adjoint).  Rate partials are
// summed per tile into a per-tile slot (same workgroup, launches in order:
// deterministic) and reduced per lattice in tile order at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"
#include "lbm_tile.hpp"

using lbm::Consts;
using lbm::TileRef;
using namespace lbm;

namespace {

constexpr int kAdjBlock = 256;
constexpr int kAdjOut = kAdjBlock - 4;

__device__ __forceinline__ int64_t wrap_in(int64_t x, int64_t n, bool small) {
  if (small) return lbm::wrap_mod(x, n);
  return x < 0 ? x + n : (x >= n ? x - n : x);
}

// Forward quantities of one node that the reverse sweep reuses.
struct NodeFwd {
  double rho, J, zeta, e, psi, eps;
  double u, s, X, T, w, ir;  // ir = 1/rho
  double e_eq, psi_eq, eps_eq;
};

template <int EQ>
__device__ __forceinline__ void node_forward(const Consts& c, double f0,
                                             double fp, double fm, double g0,
                                             double gp, double gm, NodeFwd& q) {
  const double sf = fp + fm, sg = gp + gm;
  q.rho = lbm::density(c, f0, fp, fm);
  q.J = c.mJ * (fp - fm);
  q.e = c.me * (sf - 2.0 * f0);
  q.zeta = c.mz * (g0 + sg);
  q.psi = c.mpsi * (gp - gm);
  q.eps = c.meps * (sg - 2.0 * g0);
  lbm::thermo(c, q.rho, q.J, q.zeta, q.u, q.s, q.X, q.T, q.ir);
  q.w = lbm::recip(q.T);
  if (EQ == 0 || c.eq_kind == 0) {
    const double p = q.rho * c.r * q.T;
    q.e_eq = 3.0 * (q.J * q.u + p) - c.two_l2 * q.rho;
    q.psi_eq = q.zeta * q.u;
    q.eps_eq = c.eps_c * q.rho * q.X + q.e_eq * q.s;
  } else if (c.eq_kind == 2) {
    q.e_eq = 3.0 * (q.J * q.u + lbm::iso_pressure(c, q.rho)) - c.two_l2 * q.rho;
    q.psi_eq = 0.0;
    q.eps_eq = 0.0;
  } else {
    q.e_eq = c.lin[0] * q.rho + c.lin[1] * q.J + c.lin[2] * q.zeta;
    q.psi_eq = c.lin[3] * q.rho + c.lin[4] * q.J + c.lin[5] * q.zeta;
    q.eps_eq = c.lin[6] * q.rho + c.lin[7] * q.J + c.lin[8] * q.zeta;
  }
}

// Reverse of the equilibria (iv) and of the equation of state, given the
// adjoints of e_eq, psi_eq, eps_eq and extra adjoints of u and T (from the
// source); adds to the adjoints of rho, J, zeta.  EQ = 0 compiles the
// equilibria of section 8 only; EQ = -1 selects them from c.eq_kind.
template <int EQ>
__device__ __forceinline__ void equilibria_adjoint(const Consts& c,
                                                   const NodeFwd& q, double eb,
                                                   double pb, double xb,
                                                   double ub, double Tb,
                                                   double& rb, double& Jb,
                                                   double& zb) {
  double sb = 0.0, Xb = 0.0;
  const double ir = q.ir;
  if (EQ == 0 || c.eq_kind == 0) {
    // eps_eq = eps_c rho X + e_eq s
    rb += c.eps_c * q.X * xb;
    Xb += c.eps_c * q.rho * xb;
    eb += q.s * xb;
    sb += q.e_eq * xb;
    // psi_eq = zeta u
    zb += q.u * pb;
    ub += q.zeta * pb;
    // e_eq = 3 (J u + p) - 2 lambda^2 rho, p = rho r T
    Jb += 3.0 * q.u * eb;
    ub += 3.0 * q.J * eb;
    const double pbar = 3.0 * eb;
    rb -= c.two_l2 * eb;
    rb += c.r * q.T * pbar;
    Tb += q.rho * c.r * pbar;
  } else if (c.eq_kind == 2) {
    // e_eq = 3 (J u + p_iso) - 2 lambda^2 rho, d p_iso / d rho = gamma p_iso / rho
    Jb += 3.0 * q.u * eb;
    ub += 3.0 * q.J * eb;
    rb += (3.0 * c.gamma * lbm::iso_pressure(c, q.rho) * ir - c.two_l2) * eb;
  } else {
    rb += c.lin[0] * eb + c.lin[3] * pb + c.lin[6] * xb;
    Jb += c.lin[1] * eb + c.lin[4] * pb + c.lin[7] * xb;
    zb += c.lin[2] * eb + c.lin[5] * pb + c.lin[8] * xb;
  }
  // T = T0 exp(X), X = (gamma-1) ln(rho/rho0) + gamma s / cp - gamma s0 / cp
  Xb += q.T * Tb;
  rb += c.gm1 * ir * Xb;
  sb += c.gcp * Xb;
  // u = J / rho, s = zeta / rho
  Jb += ub * ir;
  rb -= q.u * ub * ir;
  zb += sb * ir;
  rb -= q.s * sb * ir;
}

// Sum of v over the 64 lanes of the wavefront (xor butterfly); lane 0's
// result has a fixed summation order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__global__ __launch_bounds__(kAdjBlock) void k_adjoint_step(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const TileRef* __restrict__ tiles, int64_t ntiles,
    const double* __restrict__ f, const double* __restrict__ fbn,
    double* __restrict__ fbo, int64_t S, double* __restrict__ rslots) {
  __shared__ double su[kAdjBlock], sT[kAdjBlock], sA[kAdjBlock], sB[kAdjBlock];
  __shared__ double wsum[3][kAdjBlock / 64];
  const int64_t b = blockIdx.x;
  if (b >= ntiles) return;  // uniform over the workgroup
  const TileRef tr = tiles[b];
  const int64_t off = offs[tr.inst];
  const int64_t n = offs[tr.inst + 1] - off;
  const Consts c = cs[tr.inst];
  const int t = threadIdx.x;
  const bool small = n < kAdjBlock + 4;
  const int64_t jl0 = (int64_t)tr.t * kAdjOut - 2 + t;
  const int64_t j = wrap_in(jl0, n, small);
  const int64_t jr = j + 1 == n ? 0 : j + 1;
  const int64_t jm = j == 0 ? n - 1 : j - 1;
  const double* F = f + off;
  const double* B = fbn + off;
  // Phase A: forward recomputation at the node, streamed adjoint.
  NodeFwd q;
  node_forward<-1>(c, F[j], F[S + j], F[2 * S + j], F[3 * S + j], F[4 * S + j],
                   F[5 * S + j], q);
  su[t] = q.u;
  sT[t] = q.T;
  const double a0 = B[j], ap = B[S + jr], am = B[2 * S + jm];
  const double b0 = B[3 * S + j], bp = B[4 * S + jr], bm = B[5 * S + jm];
  __syncthreads();
  // Phase B: the node's source term and what it sends to its neighbours.
  double du = 0.0, dT = 0.0;
  const double Zb = c.ga * (b0 + bp + bm);  // adjoint of zeta + dz
  if (t >= 1 && t < kAdjBlock - 1) {
    du = su[t + 1] - su[t - 1];
    dT = sT[t + 1] - sT[t - 1];
    sA[t] = 2.0 * c.src_c * q.rho * q.w * du * Zb;
    sB[t] = 2.0 * c.src_c * c.cPr * q.rho * q.w * q.w * dT * Zb;
  }
  __syncthreads();
  const bool own = t >= 2 && t < kAdjBlock - 2 && jl0 < n;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if (own) {
    const double Q = du * du + c.cPr * dT * dT * q.w;
    double ub = sA[t - 1] - sA[t + 1];
    double Tb = sB[t - 1] - sB[t + 1] -
                Zb * c.src_c * q.rho * q.w * q.w *
                    (du * du + 2.0 * c.cPr * dT * dT * q.w);
    double rb = Zb * c.src_c * q.w * Q;
    if (c.src_c != 0.0) r0 -= Zb * 0.25 * q.rho * q.w * Q * c.ise2;
    // (vi)^T: adjoints of (rho, J, zeta, e*, psi*, eps*) from fbar*
    rb += c.fa * (a0 + ap + am);
    double Jb = c.fc * (ap - am);
    const double esb = c.fb * (0.5 * (ap + am) - a0);
    double zb = Zb;
    const double psisb = c.gc * (bp - bm);
    const double epssb = c.gb * (0.5 * (bp + bm) - b0);
    // (v)^T
    const double eb = (1.0 - c.s_e) * esb;
    const double psib = (1.0 - c.s_psi) * psisb;
    const double epsb = (1.0 - c.s_eps) * epssb;
    r0 += (q.e_eq - q.e) * esb;
    r1 += (q.psi_eq - q.psi) * psisb;
    r2 += (q.eps_eq - q.eps) * epssb;
    // (iv)^T and the equation of state
    equilibria_adjoint<-1>(c, q, c.s_e * esb, c.s_psi * psisb, c.s_eps * epssb,
                           ub, Tb, rb, Jb, zb);
    // (ii)^T: fbar(t) = M^T mbar
    double* O = fbo + off;
    O[j] = c.rho0 * rb - 2.0 * c.me * eb;
    O[S + j] = c.rho0 * rb + c.mJ * Jb + c.me * eb;
    O[2 * S + j] = c.rho0 * rb - c.mJ * Jb + c.me * eb;
    O[3 * S + j] = c.mz * zb - 2.0 * c.meps * epsb;
    O[4 * S + j] = c.mz * zb + c.mpsi * psib + c.meps * epsb;
    O[5 * S + j] = c.mz * zb - c.mpsi * psib + c.meps * epsb;
  }
  // rate partials: a butterfly sum inside each wavefront (lane 0's total,
  // a fixed order), then the wavefronts' totals in order
  r0 = wave_sum(r0);
  r1 = wave_sum(r1);
  r2 = wave_sum(r2);
  if ((t & 63) == 0) {
    wsum[0][t >> 6] = r0;
    wsum[1][t >> 6] = r1;
    wsum[2][t >> 6] = r2;
  }
  __syncthreads();
  if (t < 3) {
    double a = wsum[t][0];
    for (int w = 1; w < kAdjBlock / 64; ++w) a += wsum[t][w];
    rslots[3 * b + t] += a;
  }
}

// ------------------------------------------------ register-tile adjoint --
//
// K reverse steps of a tile per launch, on its own tile table (halo H = 2K
// on each side, or 2K + 2 when only every second forward state is stored, K
// the forward's steps per launch).  The tile has the forward kernels'
// layout: WG wavefronts, lane l of wavefront w holding the P consecutive
// nodes from tile index 62 P w + P l, so that neighbouring wavefronts share
// two lanes (lane 0 of w mirrors lane 62 of w - 1, lane 63 of w mirrors
// lane 1 of w + 1) and a tile spans P (62 WG + 2) nodes.  fbar stays in
// registers; each step takes the forward state f(t) of the tile (coalesced
// loads issued during the previous step, through LDS, or recomputed from the
// stored state before: see k_adjoint_tile) and does, with neighbours inside
// the wavefront through DPP only:
//   A  u, T (and rho, s, X) of every node from f(t);
//   -  streamed adjoint: fbar*_+(k) = fbar_+(k+1), fbar*_-(k) = fbar_-(k-1);
//   B  each node's source adjoint zbar and the terms it sends its neighbours,
//      A_k = 2 c rho w du zbar and B_k = 2 c (cp/Pr) rho w^2 dT zbar;
//   C  the gather of A, B from both neighbours and the node-local chain.
// One step has radius 2 in fbar(t+1) and f(t), so the wrong values the
// outermost lanes get from their missing neighbours reach two nodes into
// the wavefront: the mirror lanes (P >= 2 nodes) absorb them, and before
// every step the mirror lanes take fbar (and a recomputed f(t)) from the
// lanes they mirror, through LDS with one workgroup barrier.  Rate partials
// are summed over the tile's output nodes [H, W - H) that the wavefront owns
// (the output regions of the tiles partition each lattice).
template <int P>
__device__ __forceinline__ void shift_left(double (&a)[P], double in_right) {
#pragma unroll
  for (int k = 0; k < P - 1; ++k) a[k] = a[k + 1];
  a[P - 1] = in_right;
}
template <int P>
__device__ __forceinline__ void shift_right(double (&a)[P], double in_left) {
#pragma unroll
  for (int k = P - 1; k > 0; --k) a[k] = a[k - 1];
  a[0] = in_left;
}

// One reverse step of a lane's P nodes in the forward step's own scaled
// variables (collide_local: rh = f0 + f+ + f-, Jh = f+ - f-, zh = g0 + g+ +
// g-, uh, sh, X, Th; the populations and their adjoints are the same in
// both).  The forward at a node, before streaming:
//   d = jup - (f+ + f-), jup = Jh uh + hP rh Th (section 8; jup with the
//     isentropic pressure for eq_kind 2), or d = eh - (f+ + f- - 2 f0)
//     with linear eh (eq_kind 1);
//   f0 -= s_e d, f+- += s_e d / 2 (s_e / 3, s_e / 6 for eq_kind 1);
//   dpr = psih - (g+ - g-), dxr = epsh - (g+ + g- - 2 g0);
//   g0 += -s_eps dxr / 3 + add, g+- += +-s_psi dpr / 2 + s_eps dxr / 6 + add,
//   add = hS rh w (du^2 + hC dT^2 w), w = 1 / Th, du, dT across j-1, j+1.
// Given a = fbar*(f), b = fbar*(g) at the node (after the transposed
// streaming) the reverse is
//   db = s_e (a+ + a-)/2 - s_e a0, dprb = s_psi (b+ - b-) / 2,
//   dxrb = s_eps ((b+ + b-)/2 - b0) / 3, addb = b0 + b+ + b-,
// the adjoints of the equilibria from (db, dprb, dxrb), of the source from
// addb (its terms in the neighbours' uh, Th are gathered as A, B), of the
// thermodynamic state (X = (gamma-1) ln rh + gamma sh + xs0, Th = e^X,
// uh = Jh / rh, sh = zh / rh) and of the moments back to the populations,
// plus the direct paths of the relaxation.  Rate partials: d db / s_e,
// dpr (b+ - b-) / 2, dxr ((b+ + b-)/2 - b0) / 3, and the source's
// d hS / d s_e, accumulated without their constant factors over the
// owned nodes: acc = {sum d E1, sum F Q, sum dpr (b+ - b-), sum dxr E2}
// (see rate_partials).  PRE: the thermodynamic state of f(t) is given in pre[k]
// (kept by the forward step that recomputed the next state from f(t): the
// same arithmetic on the same populations, so the same bits).
template <int P, int EQ, bool PRE = false>
__device__ __forceinline__ void adjoint_step_local(
    const Consts& c, const double (&ft)[6][P], double (&fb)[6][P],
    const bool (&own)[P], double (&acc)[4], const lbm::NodeThermo* pre = nullptr) {
#pragma clang fp contract(off)
  // A: scaled moments and thermodynamic state of every node of f(t)
  double rh[P], uh[P], sh[P], X[P], Th[P], ir[P], lr[P], w[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    rh[k] = (ft[0][k] + ft[1][k]) + ft[2][k];
    if constexpr (PRE) {
      uh[k] = pre[k].uh;
      sh[k] = pre[k].sh;
      X[k] = pre[k].X;
      Th[k] = pre[k].Th;
      lr[k] = pre[k].lr;
      ir[k] = pre[k].ir;
      w[k] = pre[k].w;
    } else {
      const double Jh = ft[1][k] - ft[2][k];
      const double zh = ft[3][k] + (ft[4][k] + ft[5][k]);
      lbm::thermo_scaled(c, rh[k], Jh, zh, uh[k], sh[k], X[k], Th[k], lr[k], ir[k]);
    }
  }
  const double fpR = lbm::from_right(fb[1][0]), gpR = lbm::from_right(fb[4][0]);
  const double fmL = lbm::from_left(fb[2][P - 1]), gmL = lbm::from_left(fb[5][P - 1]);
  const double uL = lbm::from_left(uh[P - 1]), TL = lbm::from_left(Th[P - 1]);
  const double uR = lbm::from_right(uh[0]), TR = lbm::from_right(Th[0]);
  // streamed adjoint (transpose of (viii)): fb now holds fbar*
  shift_left<P>(fb[1], fpR);
  shift_left<P>(fb[4], gpR);
  shift_right<P>(fb[2], fmL);
  shift_right<P>(fb[5], gmL);
  // B: the source's adjoint factor F = hS rh w addb of each node, and what
  // it sends its neighbours: A = 2 F du (to uh), B = 2 F hC w dT (to Th)
  double A[P], B[P], F[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const double ul = k == 0 ? uL : uh[k - 1], ur = k == P - 1 ? uR : uh[k + 1];
    const double tl = k == 0 ? TL : Th[k - 1], tr = k == P - 1 ? TR : Th[k + 1];
    if constexpr (!PRE) w[k] = lbm::recip(Th[k]);
    const double addb = (fb[3][k] + fb[4][k]) + fb[5][k];
    F[k] = (c.hS * (rh[k] * w[k])) * addb;
    const double F2 = F[k] + F[k];
    A[k] = F2 * (ur - ul);
    B[k] = ((F2 * c.hC) * w[k]) * (tr - tl);
  }
  const double AL = lbm::from_left(A[P - 1]), BL = lbm::from_left(B[P - 1]);
  const double AR = lbm::from_right(A[0]), BR = lbm::from_right(B[0]);
  // C: gather and node-local reverse chain
#pragma unroll
  for (int k = 0; k < P; ++k) {
    __builtin_amdgcn_sched_barrier(0);
    const double ul = k == 0 ? uL : uh[k - 1], ur = k == P - 1 ? uR : uh[k + 1];
    const double tl = k == 0 ? TL : Th[k - 1], tr = k == P - 1 ? TR : Th[k + 1];
    const double al = k == 0 ? AL : A[k - 1], ar = k == P - 1 ? AR : A[k + 1];
    const double bl = k == 0 ? BL : B[k - 1], br = k == P - 1 ? BR : B[k + 1];
    const double f0 = ft[0][k], fp = ft[1][k], fm = ft[2][k];
    const double g0 = ft[3][k], gp = ft[4][k], gm = ft[5][k];
    const double a0 = fb[0][k], ap = fb[1][k], am = fb[2][k];
    const double b0 = fb[3][k], bp = fb[4][k], bm = fb[5][k];
    const double r = rh[k], u = uh[k], sv = sh[k], x = X[k], T = Th[k];
    const double Jh = fp - fm, sf = fp + fm, sg = gp + gm, zh = g0 + sg;
    // adjoints of the relaxation's increments
    const double E1 = fma(0.5, ap + am, -a0);
    const double E2 = fma(0.5, bp + bm, -b0);
    const double bd = bp - bm;
    const double dprb = c.sp_2 * bd;
    const double dxrb = c.sx_3 * E2;
    // the forward's equilibria, increments and the adjoints of the
    // equilibria: rhb, Jhb, zhb, uhb, Thb, shb, Xb, lrb
    double d, db, psih, epsh;
    double rhb, Jhb, zhb = 0.0, uhb = 0.0, Thb = 0.0, shb = 0.0, Xb = 0.0, lrb = 0.0;
    if (EQ == 0 || c.eq_kind == 0) {
      const double hPr = c.hP * r;
      const double jup = fma(Jh, u, hPr * T);
      const double eh = fma(-2.0, r, 3.0 * jup);
      psih = zh * u;
      const double tgr = c.two_g * r;
      epsh = fma(eh, sv, tgr * x);
      d = jup - sf;
      db = c.s_e * E1;
      // epsh = eh sh + (2/gamma) rh X, psih = zh uh, eh = 3 jup - 2 rh,
      // jup = Jh uh + hP rh Th
      const double ehb = sv * dxrb;
      shb = eh * dxrb;
      Xb = tgr * dxrb;
      zhb = u * dprb;
      const double jupb = fma(3.0, ehb, db);
      rhb = fma(-2.0, ehb, (c.two_g * x) * dxrb);
      rhb = fma(c.hP * T, jupb, rhb);
      Jhb = u * jupb;
      uhb = fma(Jh, jupb, zh * dprb);
      Thb = hPr * jupb;
    } else if (c.eq_kind == 2) {
      const double pe = lbm::exp_fin(c.gm1 * lr[k]);
      const double hPr = c.hP * r;
      const double jup = fma(Jh, u, hPr * pe);
      psih = 0.0;
      epsh = 0.0;
      d = jup - sf;
      db = c.s_e * E1;
      rhb = (c.hP * pe) * db;
      lrb = (c.gm1 * (hPr * pe)) * db;
      Jhb = u * db;
      uhb = Jh * db;
    } else {
      const double eh = fma(c.hlin[2], zh, fma(c.hlin[1], Jh, c.hlin[0] * r));
      psih = fma(c.hlin[5], zh, fma(c.hlin[4], Jh, c.hlin[3] * r));
      epsh = fma(c.hlin[8], zh, fma(c.hlin[7], Jh, c.hlin[6] * r));
      d = eh - fma(-2.0, f0, sf);
      db = c.se_3 * E1;
      rhb = fma(c.hlin[6], dxrb, fma(c.hlin[3], dprb, c.hlin[0] * db));
      Jhb = fma(c.hlin[7], dxrb, fma(c.hlin[4], dprb, c.hlin[1] * db));
      zhb = fma(c.hlin[8], dxrb, fma(c.hlin[5], dprb, c.hlin[2] * db));
    }
    // the source at this node (add = hS rh w Q, Q = du^2 + hC dT^2 w) and
    // the neighbours' terms in this node's uh and Th
    const double du = ur - ul, dT = tr - tl;
    const double tw = (c.hC * (dT * dT)) * w[k];
    const double Q = fma(du, du, tw);
    const double addb = (b0 + bp) + bm;
    rhb = fma((c.hS * w[k]) * addb, Q, rhb);
    // d add / d w = hS rh (Q + tw), d w / d Th = -w^2, F = hS rh w addb
    Thb = fma(-w[k], F[k] * (Q + tw), Thb);
    uhb += al - ar;
    Thb += bl - br;
    if (own[k]) {
      acc[0] = fma(d, E1, acc[0]);
      acc[1] = fma(F[k], Q, acc[1]);
      acc[2] = fma(psih - (gp - gm), bd, acc[2]);
      acc[3] = fma(epsh - fma(-2.0, g0, sg), E2, acc[3]);
    }
    // the thermodynamic state: Th = e^X, X = gm1 lr + gamma sh + xs0,
    // lr = ln rh, uh = Jh / rh, sh = zh / rh
    Xb = fma(T, Thb, Xb);
    lrb = fma(c.gm1, Xb, lrb);
    shb = fma(c.gamma, Xb, shb);
    const double iv = ir[k];
    zhb = fma(iv, shb, zhb);
    Jhb = fma(iv, uhb, Jhb);
    rhb = fma(iv, lrb - fma(u, uhb, sv * shb), rhb);
    // the moments and the relaxation's direct paths
    const double dfm = (EQ == 0 || c.eq_kind != 1) ? a0 : fma(2.0, db, a0);
    const double rd = rhb - db, zx = zhb - dxrb;
    fb[0][k] = dfm + rhb;
    fb[1][k] = (ap + rd) + Jhb;
    fb[2][k] = (am + rd) - Jhb;
    fb[3][k] = fma(2.0, dxrb, b0) + zhb;
    fb[4][k] = (bp + zx) - dprb;
    fb[5][k] = (bm + zx) + dprb;
  }
}

// The three rate partials from the sums adjoint_step_local accumulates:
// d/ds_e = sum d E1 (x 1/3 for the linear equilibria, whose increment is
// s_e d / 3) + (d hS / d s_e) / hS sum F Q, d/ds_psi = sum dpr (b+ - b-) / 2,
// d/ds_eps = sum dxr E2 / 3.
__device__ __forceinline__ void rate_partials(const Consts& c,
                                              const double (&acc)[4],
                                              double& r0, double& r1,
                                              double& r2) {
#pragma clang fp contract(off)
  const double se = c.eq_kind == 1 ? acc[0] * (1.0 / 3.0) : acc[0];
  r0 = c.hS != 0.0 ? fma(c.hSd / c.hS, acc[1], se) : se;
  r1 = 0.5 * acc[2];
  r2 = acc[3] * (1.0 / 3.0);
}

// Mirror lanes of the reverse tile before a step: lanes 1 and 62 publish
// fbar (and, after a recomputation, f(t)) in `edge` (one buffer of a
// double-buffered pair, as in the forward kernels), then lane 0 takes lane
// 62 of the wavefront to its left and lane 63 lane 1 of the one to its
// right.  with_ft is the same for every wavefront of the workgroup.
template <int P, int WG>
__device__ __forceinline__ void adjoint_mirror_refresh(
    double (&fb)[6][P], double (&ft)[6][P], bool with_ft,
    double (*edge)[2][12 * P], int lane, int wave) {
  if (lane == 1 || lane == 62) {
    double* d = edge[wave][lane == 62];
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) d[q * P + k] = fb[q][k];
    if (with_ft) {
#pragma unroll
      for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int k = 0; k < P; ++k) d[6 * P + q * P + k] = ft[q][k];
    }
  }
  __syncthreads();
  const bool left = lane == 0 && wave > 0, right = lane == 63 && wave < WG - 1;
  if (left || right) {
    const double* e = left ? edge[wave - 1][1] : edge[wave + 1][0];
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) fb[q][k] = e[q * P + k];
    if (with_ft) {
#pragma unroll
      for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int k = 0; k < P; ++k) ft[q][k] = e[6 * P + q * P + k];
    }
  }
}

// Reverse steps i_hi-1 down to i_lo of a checkpoint segment.  E = 1: the
// forward state of every step i is stored, ck (i = 0) or seg + (i-1)*SD.
// E = 2: only the even ones are (state i at seg + (i/2-1)*SD); an odd step's
// state is recomputed from the one before (tile_step, the forward kernels'
// node arithmetic in the same order: bitwise the state they store), which
// then serves the next (even) step, so each such pair of steps loads one
// state.  The prefetch of a pair's state is issued during the previous
// pair.  If the launch's first step is odd, its recomputed state is wrong at
// the two outer nodes of each side, which costs the halo two more nodes
// (H >= 2K + 2).  EQ = 0: every lattice of the table has the equilibria of
// section 8.
template <int P, int WG, int E, int EQ>
__global__ __launch_bounds__(64 * WG) void k_adjoint_tile(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const TileRef* __restrict__ tiles, int64_t ntiles,
    const double* __restrict__ ck, const double* __restrict__ seg, int64_t SD,
    int i_lo, int i_hi, const double* __restrict__ fbn,
    double* __restrict__ fbo, int64_t S, int H, double* __restrict__ rslots) {
  static_assert(P > 1 || WG == 1, "P = 1 tiles have one wavefront");
  constexpr int WW = 64 * P;   // nodes of one wavefront
  constexpr int WS = 62 * P;   // wavefront stride in the tile
  constexpr int W = lbm::tile_nodes(P, WG);
  __shared__ double stage[WG * (WW + 64)];
  __shared__ double edge[2][WG][2][12 * P];
  __shared__ double red[3][64 * WG];
  const int64_t b = blockIdx.x;
  if (b >= ntiles) return;  // uniform over the workgroup
  const TileRef tr = tiles[b];
  const int64_t off = offs[tr.inst];
  const int64_t n = offs[tr.inst + 1] - off;
  const Consts& c = cs[tr.inst];  // loaded where used
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* lds = stage + wave * (WW + 64);
  const int OUT = W - 2 * H;
  const int64_t start = (int64_t)tr.t * OUT - H;
  const int64_t wstart = start + wave * WS;
  const bool inside = start >= 0 && start + W <= n;
  const bool small = n < W;
  // output nodes of the tile that this wavefront owns (the mirror lanes
  // belong to the neighbours)
  const bool mirror = (lane == 0 && wave > 0) || (lane == 63 && wave < WG - 1);
  bool own[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int it = wave * WS + lane * P + k;
    own[k] = !mirror && it >= H && it < W - H && start + it < n;
  }
  // the segment's global indices are the same in every state
  int64_t gi[P];
  tile_index<P>(n, wstart, inside, small, lane, gi);
  double fb[6][P], raw[6][P];
  tile_fetch<P>(fbn + off, S, gi, raw);
  tile_transpose<P>(lane, lds, raw, fb);
  auto state = [&](int i) {
    return (i == 0 ? ck : seg + (int64_t)((i - 1) / E) * SD) + off;
  };
  // the stored state step i starts from
  auto base = [](int i) { return E == 2 ? (i & ~1) : i; };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // the stored state of the next (earlier) step or pair is fetched while
  // this one computes
  tile_fetch<P>(state(base(i_hi - 1)), S, gi, raw);
  int buf = 0;
  auto refresh = [&](double (&ft)[6][P], bool recomputed) {
    if constexpr (WG > 1) {
      adjoint_mirror_refresh<P, WG>(fb, ft, recomputed, edge[buf], lane, wave);
      buf ^= 1;
    }
  };
  int i = i_hi - 1;
  if (E == 1 || !(i & 1)) {
    // E = 1: every step's state is stored; E = 2: a launch whose first step
    // is even starts with that stored state
    for (; i >= i_lo && (E == 1 || i == i_hi - 1); --i) {
      double ft[6][P];
      tile_transpose<P>(lane, lds, raw, ft);
      if (i > i_lo) tile_fetch<P>(state(base(i - 1)), S, gi, raw);
      refresh(ft, false);
      adjoint_step_local<P, EQ>(c, ft, fb, own, acc);
    }
  }
  // E = 2, pairs of steps (i odd, i - 1): state i is recomputed from the
  // stored state i - 1, whose thermodynamic state the recomputation keeps
  // for step i - 1
  for (; E == 2 && i >= i_lo; i -= 2) {
    double fa[6][P], ft[6][P];
    tile_transpose<P>(lane, lds, raw, fa);
    if (i - 2 >= i_lo) tile_fetch<P>(state(base(i - 2)), S, gi, raw);
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) ft[q][k] = fa[q][k];
    lbm::NodeThermo th[P];
    tile_step<P, EQ, true>(c, ft, th);
    refresh(ft, true);
    adjoint_step_local<P, EQ>(c, ft, fb, own, acc);
    if (i - 1 >= i_lo) {
      refresh(fa, false);
      adjoint_step_local<P, EQ, true>(c, fa, fb, own, acc, th);
    }
  }
  const int lo = max(H - wave * WS, wave > 0 ? P : 0);
  const int hi = min(W - H - wave * WS, wave < WG - 1 ? WW - P : WW);
  tile_store<P>(fbo + off, S, n, wstart, lo, hi, lane, lds, fb);
  double r0, r1, r2;
  rate_partials(c, acc, r0, r1, r2);
  const int t = threadIdx.x;
  red[0][t] = r0;
  red[1][t] = r1;
  red[2][t] = r2;
  __syncthreads();
  for (int m = 32 * WG; m > 0; m >>= 1) {
    if (t < m) {
      red[0][t] += red[0][t + m];
      red[1][t] += red[1][t + m];
      red[2][t] += red[2][t + m];
    }
    __syncthreads();
  }
  if (t < 3) rslots[3 * b + t] += red[t][0];
}

template <int P, int WG, int E, int EQ>
void launch_adjoint_tile_t(const Consts* cs, const int64_t* offs,
                           const TileRef* tiles, int64_t ntiles,
                           const double* ck, const double* seg, int64_t SD,
                           int i_lo, int i_hi, const double* fbn, double* fbo,
                           int64_t S, int H, double* rslots, hipStream_t s) {
  hipLaunchKernelGGL((k_adjoint_tile<P, WG, E, EQ>), dim3((unsigned)ntiles),
                     dim3(64 * WG), 0, s, cs, offs, tiles, ntiles, ck, seg, SD,
                     i_lo, i_hi, fbn, fbo, S, H, rslots);
}

// E: stride of the stored segment states (1, or 2 at P = 2); eq: 0 when
// every lattice has the equilibria of section 8, else -1.
int launch_adjoint_tile(int P, int WG, int E, int eq, const Consts* cs,
                        const int64_t* offs, const TileRef* tiles,
                        int64_t ntiles, const double* ck, const double* seg,
                        int64_t SD, int i_lo, int i_hi, const double* fbn,
                        double* fbo, int64_t S, int H, double* rslots,
                        hipStream_t s) {
  if (i_hi - i_lo < 1 || 2 * (i_hi - i_lo) + (E == 2 ? 2 : 0) > H ||
      2 * H >= lbm::tile_nodes(P, WG))
    return set_err(LBM_EINVAL, "bad adjoint tile geometry");
#define LBM_ADJ_CASE(PP, WW, EE)                                               \
  if (P == PP && WG == WW && E == EE) {                                        \
    if (eq == 0)                                                               \
      launch_adjoint_tile_t<PP, WW, EE, 0>(cs, offs, tiles, ntiles, ck, seg,   \
                                           SD, i_lo, i_hi, fbn, fbo, S, H,     \
                                           rslots, s);                         \
    else                                                                       \
      launch_adjoint_tile_t<PP, WW, EE, -1>(cs, offs, tiles, ntiles, ck, seg,  \
                                            SD, i_lo, i_hi, fbn, fbo, S, H,    \
                                            rslots, s);                        \
    return hip_check(hipGetLastError(), "k_adjoint_tile");                     \
  }
  LBM_ADJ_CASE(1, 1, 1)
  LBM_ADJ_CASE(2, 1, 1)
  LBM_ADJ_CASE(2, 2, 1)
  LBM_ADJ_CASE(2, 4, 1)
  LBM_ADJ_CASE(2, 8, 1)
  LBM_ADJ_CASE(2, 1, 2)
  LBM_ADJ_CASE(2, 2, 2)
  LBM_ADJ_CASE(2, 4, 2)
  LBM_ADJ_CASE(2, 8, 2)
  LBM_ADJ_CASE(4, 8, 1)  // the only P = 4 shape rev_shape gives
#undef LBM_ADJ_CASE
  return set_err(LBM_EINVAL,
                 "unsupported adjoint tile shape P=%d waves=%d stride=%d", P,
                 WG, E);
}

// fbar of the equilibrium initialisation -> adjoints of rho, J, zeta.
__global__ __launch_bounds__(256) void k_equilibrium_adjoint(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const double* __restrict__ rho, const double* __restrict__ J,
    const double* __restrict__ zeta, const double* __restrict__ fb,
    double* __restrict__ rho_b, double* __restrict__ J_b,
    double* __restrict__ zeta_b, int64_t S) {
  const int inst = blockIdx.x;
  const Consts c = cs[inst];
  for (int64_t j = offs[inst] + threadIdx.x; j < offs[inst + 1]; j += 256) {
    NodeFwd q;
    q.rho = rho[j];
    q.J = J[j];
    q.zeta = zeta[j];
    lbm::thermo(c, q.rho, q.J, q.zeta, q.u, q.s, q.X, q.T, q.ir);
    if (c.eq_kind == 0) {
      const double p = q.rho * c.r * q.T;
      q.e_eq = 3.0 * (q.J * q.u + p) - c.two_l2 * q.rho;
    }
    const double a0 = fb[j], ap = fb[S + j], am = fb[2 * S + j];
    const double b0 = fb[3 * S + j], bp = fb[4 * S + j], bm = fb[5 * S + j];
    double rb = c.fa * (a0 + ap + am);
    double Jb = c.fc * (ap - am);
    double zb = c.ga * (b0 + bp + bm);
    const double eb = c.fb * (0.5 * (ap + am) - a0);
    const double pb = c.gc * (bp - bm);
    const double xb = c.gb * (0.5 * (bp + bm) - b0);
    equilibria_adjoint<-1>(c, q, eb, pb, xb, 0.0, 0.0, rb, Jb, zb);
    rho_b[j] = rb;
    J_b[j] = Jb;
    zeta_b[j] = zb;
  }
}

// fbar = M^T mbar (mbar in moment order rho, J, zeta, e, psi, eps).
__global__ __launch_bounds__(256) void k_moments_adjoint(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const double* __restrict__ mb, double* __restrict__ fb, int64_t S) {
  const int inst = blockIdx.x;
  const Consts c = cs[inst];
  for (int64_t j = offs[inst] + threadIdx.x; j < offs[inst + 1]; j += 256) {
    const double rb = mb[j], Jb = mb[S + j], zb = mb[2 * S + j];
    const double eb = mb[3 * S + j], pb = mb[4 * S + j], xb = mb[5 * S + j];
    fb[j] = c.rho0 * rb - 2.0 * c.me * eb;
    fb[S + j] = c.rho0 * rb + c.mJ * Jb + c.me * eb;
    fb[2 * S + j] = c.rho0 * rb - c.mJ * Jb + c.me * eb;
    fb[3 * S + j] = c.mz * zb - 2.0 * c.meps * xb;
    fb[4 * S + j] = c.mz * zb + c.mpsi * pb + c.meps * xb;
    fb[5 * S + j] = c.mz * zb - c.mpsi * pb + c.meps * xb;
  }
}

// L_i = 1/2 sum_j (rho_j - target_j)^2 per lattice (target NULL: rho0) and
// its gradient with respect to the state; fixed tree order.
__global__ __launch_bounds__(256) void k_loss(
    const Consts* __restrict__ cs, const int64_t* __restrict__ offs,
    const double* __restrict__ f, const double* __restrict__ target,
    double* __restrict__ loss, double* __restrict__ fb, int64_t S) {
  __shared__ double red[256];
  const int inst = blockIdx.x;
  const Consts c = cs[inst];
  double acc = 0.0;
  for (int64_t j = offs[inst] + threadIdx.x; j < offs[inst + 1]; j += 256) {
    const double rho = lbm::density(c, f[j], f[S + j], f[2 * S + j]);
    const double d = rho - (target ? target[j] : c.rho0);
    acc += 0.5 * d * d;
    const double g = c.rho0 * d;
    fb[j] = g;
    fb[S + j] = g;
    fb[2 * S + j] = g;
    fb[3 * S + j] = 0.0;
    fb[4 * S + j] = 0.0;
    fb[5 * S + j] = 0.0;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[inst] = red[0];
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// rbar[3*inst + q] = sum over the lattice's adjoint tiles, in tile order.
__global__ void k_rbar_reduce(const int64_t* __restrict__ first,
                              int64_t n_inst, const double* __restrict__ slots,
                              double* __restrict__ rbar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t t = first[i]; t < first[i + 1]; ++t) {
    a += slots[3 * t];
    b += slots[3 * t + 1];
    c += slots[3 * t + 2];
  }
  rbar[3 * i] = a;
  rbar[3 * i + 1] = b;
  rbar[3 * i + 2] = c;
}

// ------------------------------------------------------------ host side --

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct AdjLayout {
  int64_t n_fwd, n_rec, n_rev, n_adj, n_ck, n_seg, seg_bufs;
  size_t consts, offs, fwd_tiles, rec_tiles, rev_tiles, adj_tiles, adj_first,
      rev_first,
      rslots, scratch, pp, ckpt, seg, total;
};

// The recompute runs with the forward tile shape.
lbm_tuning rec_tuning(const lbm_tuning& t) { return t; }

// Tile shape of the checkpointed forward run.
lbm_tuning fwd_tuning(const lbm_batch* b) { return b->tune; }

// Tile shape of the blocked reverse kernel for a forward tuning and a stride
// E of the stored segment states.  Its tiles span P (62 W + 2) nodes
// (neighbouring wavefronts share two lanes) with halo H = 2K, or 2K + 2 at
// E = 2 (see k_adjoint_tile).  P = 2 keeps two wavefronts per SIMD (the
// reverse step needs 183-241 VGPRs at P = 2, over 256 at P = 4), with the
// wavefronts that give about the forward tile's width, at least the
// forward's and at most 4: two workgroups per CU, so that one computes while
// the other waits at a step's barrier (measured with the earlier two
// barriers per step: the 1024-lattice gradient's reverse phase took 442 ms
// at 4 wavefronts, 472 at 8, 512 at 2); a halo too wide for those tiles
// falls back to P = 4 with 8 wavefronts and E = 1.  A forward of one node
// per lane (small problems) keeps P = 1, W = 1, E = 1 (about 110 VGPRs).
struct RevShape {
  int P, W, H, E;
  int64_t out() const { return (int64_t)tile_nodes(P, W) - 2 * (int64_t)H; }
};

RevShape rev_shape(const lbm_tuning& t, int E) {
  const int K = t.steps_per_launch;
  // one node per lane (small lattices, bound by each step's latency): the
  // same for the reverse, whose halo the forward's K already fits
  if (t.nodes_per_lane == 1) return RevShape{1, 1, 2 * K, 1};
  RevShape r{2, std::min(4, std::max(t.waves_per_group,
                                     t.nodes_per_lane * t.waves_per_group / 2)),
             2 * K + (E == 2 ? 2 : 0), E};
  if (2 * r.H >= tile_nodes(2, r.W)) r = RevShape{4, 8, 2 * K, 1};
  return r;
}

// Tiles of `out` output nodes covering every lattice (0 if out < 1: such a
// shape is refused before any table is built).
int64_t tiles_of(const lbm_batch* b, int64_t out) {
  if (out < 1) return 0;
  int64_t s = 0;
  for (int64_t i = 0; i < b->n_inst; ++i)
    s += (b->offsets[i + 1] - b->offsets[i] + out - 1) / out;
  return s;
}

int64_t adj_tile_count(const lbm_batch* b) {
  int64_t s = 0;
  for (int64_t i = 0; i < b->n_inst; ++i)
    s += (b->offsets[i + 1] - b->offsets[i] + kAdjOut - 1) / kAdjOut;
  return s;
}

// Whether the reverse sweep of the batch's current settings runs one step
// per launch (LBM_KERNEL_AUTO: the blocked kernel wherever its tiles can hold
// the forward halo).
bool resolve_adj_plain(const lbm_batch* b) {
  return b->adj_kernel == LBM_KERNEL_PLAIN ||
         (b->adj_kernel == LBM_KERNEL_AUTO && rev_shape(b->tune, 1).out() < 1);
}

// Launches of the blocked reverse kernel fill the chip when they have at
// least the 2048 wavefronts that 256 CUs hold at two per SIMD.
bool rev_fills_chip(const lbm_batch* b, const RevShape& r) {
  return tiles_of(b, r.out()) * r.W >= 2048;
}

// Stride of the segment states the reverse sweep stores.  Every second one
// (the kernel recomputes the others: one forward step per pair of reverse
// steps in place of storing and loading 48 bytes per node, and half the
// segment buffer) needs the blocked kernel at P = 2 with K >= 2.  Automatic
// (0): there, where its launches fill the chip; a launch-bound sweep (small
// lattices) keeps every state, as the recomputation would lengthen each
// launch.
int resolve_every(const lbm_batch* b, bool plain) {
  if (plain || b->tune.steps_per_launch < 2) return 1;
  const RevShape r = rev_shape(b->tune, 2);
  if (r.E != 2 || r.out() < 1) return 1;
  if (b->rec_stride == 1 || b->rec_stride == 2) return b->rec_stride;
  return rev_fills_chip(b, r) ? 2 : 1;
}

// The reverse sweep's settings: one-step kernel or the blocked one with its
// tile shape and state stride, and whether the sweep overlaps the recompute
// of one checkpoint segment with the reverse steps of the next (two buffers
// of segment states): with the blocked kernel when its launches leave most
// of the chip idle, as on small lattices bound by launch latency.  A launch
// that fills the chip gains nothing from a second stream (measured on the
// 1024-lattice gradient) and the second buffer would cost its states again.
struct AdjPlan {
  bool plain, pipelined;
  RevShape rev;
};

AdjPlan adj_plan(const lbm_batch* b, bool plain, int every) {
  AdjPlan p{plain, false, rev_shape(b->tune, plain ? 1 : every)};
  p.pipelined = !plain && p.rev.out() >= 1 && !rev_fills_chip(b, p.rev);
  return p;
}

// The plan of the current settings (workspace queries) and the one that
// lbm_batch_forward_ckpt resolved (the reverse sweep and its checks).
AdjPlan current_plan(const lbm_batch* b) {
  const bool plain = resolve_adj_plain(b);
  return adj_plan(b, plain, resolve_every(b, plain));
}
AdjPlan resolved_plan(const lbm_batch* b) {
  return adj_plan(b, b->adj_plain, b->adj_every);
}

// Workspace layout.  The segment states come last: the other offsets do not
// depend on them.
AdjLayout adj_layout(const lbm_batch* b, int64_t nsteps, int64_t C,
                     const AdjPlan& P) {
  AdjLayout L{};
  L.n_fwd = b->count_tiles(fwd_tuning(b));
  L.n_rec = b->count_tiles(rec_tuning(b->tune));
  L.n_rev = tiles_of(b, P.rev.out());
  L.n_adj = adj_tile_count(b);
  L.n_ck = nsteps > 0 ? (nsteps + C - 1) / C : 1;
  // states 1 .. len-1 of a segment of len steps, or the even ones
  L.n_seg = std::max<int64_t>(0, std::min(C, nsteps) - 1) /
            (P.plain ? 1 : P.rev.E);
  const size_t state = sizeof(double) * 6 * (size_t)b->n_total;
  size_t o = 0;
  L.consts = o;
  o = align256(o + sizeof(Consts) * b->n_inst);
  L.offs = o;
  o = align256(o + sizeof(int64_t) * (b->n_inst + 1));
  L.fwd_tiles = o;
  o = align256(o + sizeof(TileRef) * std::max<int64_t>(1, L.n_fwd));
  L.rec_tiles = o;
  o = align256(o + sizeof(TileRef) * std::max<int64_t>(1, L.n_rec));
  L.rev_tiles = o;
  o = align256(o + sizeof(TileRef) * std::max<int64_t>(1, L.n_rev));
  L.adj_tiles = o;
  o = align256(o + sizeof(TileRef) * std::max<int64_t>(1, L.n_adj));
  L.adj_first = o;
  o = align256(o + sizeof(int64_t) * (b->n_inst + 1));
  L.rev_first = o;
  o = align256(o + sizeof(int64_t) * (b->n_inst + 1));
  L.rslots = o;
  o = align256(o + sizeof(double) * 3 *
                       std::max<int64_t>(1, std::max(L.n_adj, L.n_rev)));
  L.scratch = o;  // per-lattice loss / rbar staging
  o = align256(o + sizeof(double) * 3 * b->n_inst);
  L.pp = o;
  o = align256(o + state);
  L.ckpt = o;
  o = align256(o + state * (size_t)L.n_ck);
  L.seg = o;
  L.seg_bufs = P.pipelined ? 2 : 1;
  o = align256(o + state * (size_t)L.n_seg * L.seg_bufs);
  L.total = o;
  return L;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

std::vector<TileRef> tile_table(const lbm_batch* b, int64_t out) {
  std::vector<TileRef> v;
  if (out < 1) return v;
  for (int64_t i = 0; i < b->n_inst; ++i) {
    const int64_t n = b->offsets[i + 1] - b->offsets[i];
    for (int64_t t = 0; t * out < n; ++t) v.push_back(TileRef{(int32_t)i, (int32_t)t});
  }
  return v;
}

// Launches `steps` forward steps on f with ping-pong through pp (an even
// number of launches when steps >= 2; otherwise one launch and a copy).
int fwd_steps(lbm_batch* b, const Consts* cs, const int64_t* offs,
              const TileRef* tiles, int64_t ntiles, double* f, double* pp,
              int64_t steps, hipStream_t s) {
  double* a = f;
  double* w = pp;
  int64_t launches = 0;
  const lbm_tuning t = fwd_tuning(b);
  const int H = 2 * t.steps_per_launch;
  for (int k : split_steps(steps, t.steps_per_launch)) {
    int rc = launch_batch_tile(cs, offs, tiles, ntiles, a, w, b->n_total,
                               t.nodes_per_lane, H, k, t.waves_per_group,
                               b->eq_class(), s);
    if (rc) return rc;
    std::swap(a, w);
    ++launches;
  }
  if (launches & 1)
    return hip_check(hipMemcpyAsync(f, pp, sizeof(double) * 6 * b->n_total,
                                    hipMemcpyDeviceToDevice, s),
                     "hipMemcpyAsync");
  return LBM_OK;
}

// The checkpointed forward on stream s: checkpoint k is the state at step
// k * C, then the segment's launches.
int enqueue_forward_ckpt(lbm_batch* b, void* ws, double* f, int64_t nsteps,
                         int64_t C, const AdjLayout& L, hipStream_t s) {
  const size_t SB = sizeof(double) * 6 * b->n_total;
  const Consts* cs = at<Consts>(ws, L.consts);
  const int64_t* offs = at<int64_t>(ws, L.offs);
  int rc = LBM_OK;
  for (int64_t k = 0; k < L.n_ck && !rc; ++k) {
    rc = hip_check(hipMemcpyAsync(at<char>(ws, L.ckpt) + SB * k, f, SB,
                                  hipMemcpyDeviceToDevice, s),
                   "hipMemcpyAsync");
    const int64_t len = std::min(C, nsteps - k * C);
    if (!rc && len > 0)
      rc = fwd_steps(b, cs, offs, at<TileRef>(ws, L.fwd_tiles), L.n_fwd, f,
                     at<double>(ws, L.pp), len, s);
  }
  return rc;
}

int check_adj(const lbm_batch* b, const void* ws, size_t ws_bytes,
              int64_t nsteps, int64_t C) {
  if (!b || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (b->adj_ws != ws || b->adj_nsteps != nsteps || b->adj_ckpt != C ||
      !same_tuning(b->adj_tune, b->tune) || b->adj_plain_up != b->adj_plain ||
      b->adj_every_up != b->adj_every)
    return set_err(LBM_EINVAL,
                   "no checkpoints for this workspace, nsteps and ckpt_every: "
                   "call lbm_batch_forward_ckpt first");
  if (ws_bytes < adj_layout(b, nsteps, C, resolved_plan(b)).total)
    return set_err(LBM_EWORKSPACE, "adjoint workspace too small");
  return LBM_OK;
}

// The reverse sweep: recompute each checkpoint segment, then adjoint steps.
int enqueue_adjoint(lbm_batch* b, void* ws, int64_t nsteps, int64_t C,
                    double* fbar, double* rbar, hipStream_t s) {
  const AdjPlan plan = resolved_plan(b);
  const AdjLayout L = adj_layout(b, nsteps, C, plan);
  const Consts* cs = at<Consts>(ws, L.consts);
  const int64_t* offs = at<int64_t>(ws, L.offs);
  const size_t SD = 6 * (size_t)b->n_total;
  double* slots = at<double>(ws, L.rslots);
  const int64_t nsl = 3 * std::max<int64_t>(1, std::max(L.n_adj, L.n_rev));
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((nsl + 255) / 256)), dim3(256), 0,
                     s, slots, nsl, 0.0);
  int rc = hip_check(hipGetLastError(), "k_fill");
  if (rc) return rc;
  double* cur = fbar;
  double* oth = at<double>(ws, L.pp);
  const lbm_tuning rt = rec_tuning(b->tune);
  const int Prec = rt.nodes_per_lane, Wrec = rt.waves_per_group;
  const int Krec = b->tune.steps_per_launch;
  // stride of the stored segment states
  const int E = plan.plain ? 1 : plan.rev.E;
  auto seg_len = [&](int64_t k) { return std::min(C, nsteps - k * C); };
  auto ckpt = [&](int64_t k) { return at<double>(ws, L.ckpt) + SD * k; };
  // segment k's stored states (t0+1 .. t0+len-1, or the even ones) live in
  // segment buffer k % seg_bufs
  auto segbuf = [&](int64_t k) {
    return at<double>(ws, L.seg) + SD * (size_t)L.n_seg * (size_t)(k % L.seg_bufs);
  };
  auto state = [&](int64_t k, int64_t i) {
    return i == 0 ? ckpt(k) : segbuf(k) + SD * ((i - 1) / E);
  };
  // recompute of segment k on stream st: up to Krec states per launch, each
  // launch starting from a stored state (an even one at E = 2)
  const int Kst = E == 2 ? Krec & ~1 : Krec;
  if (Kst < 1)  // resolve_every gives E = 2 only for K >= 2
    return set_err(LBM_EINVAL, "recompute stride %d with K = %d", E, Krec);
  auto recompute = [&](int64_t k, hipStream_t st) -> int {
    const int64_t len = seg_len(k);
    for (int64_t i0 = 0; i0 + 1 < len; i0 += Kst) {
      const int kk = (int)std::min<int64_t>(Kst, len - 1 - i0);
      const int r = launch_batch_tile(cs, offs, at<TileRef>(ws, L.rec_tiles),
                                      L.n_rec, state(k, i0), segbuf(k),
                                      b->n_total, Prec, 2 * Krec, kk, Wrec,
                                      b->eq_class(), st, (int64_t)SD, (int)i0,
                                      E);
      if (r) return r;
    }
    return LBM_OK;
  };
  const RevShape rv = plan.rev;
  // the blocked reverse steps of segment k on s, up to Krec per launch
  auto reverse = [&](int64_t k) -> int {
    for (int64_t hi = seg_len(k); hi > 0;) {
      const int64_t lo = std::max<int64_t>(0, hi - Krec);
      const int r = launch_adjoint_tile(
          rv.P, rv.W, rv.E, b->eq_class(), cs, offs,
          at<TileRef>(ws, L.rev_tiles), L.n_rev,
          ckpt(k), segbuf(k), (int64_t)SD, (int)lo, (int)hi, cur, oth,
          b->n_total, rv.H, slots, s);
      if (r) return r;
      std::swap(cur, oth);
      hi = lo;
    }
    return LBM_OK;
  };
  if (b->adj_plain) {
    for (int64_t k = L.n_ck - 1; k >= 0; --k) {
      if ((rc = recompute(k, s))) return rc;
      for (int64_t i = seg_len(k) - 1; i >= 0; --i) {
        hipLaunchKernelGGL(k_adjoint_step, dim3((unsigned)L.n_adj),
                           dim3(kAdjBlock), 0, s, cs, offs,
                           at<TileRef>(ws, L.adj_tiles), L.n_adj,
                           (const double*)state(k, i), (const double*)cur, oth,
                           b->n_total, slots);
        if ((rc = hip_check(hipGetLastError(), "k_adjoint_step"))) return rc;
        std::swap(cur, oth);
      }
    }
  } else if (L.seg_bufs == 1) {
    for (int64_t k = L.n_ck - 1; k >= 0; --k) {
      if ((rc = recompute(k, s))) return rc;
      if ((rc = reverse(k))) return rc;
    }
  } else {
    // Pipelined: segment k-1 is recomputed on the side stream while the
    // reverse steps of segment k run on s.  Segment buffer k % 2 is written
    // by recompute(k) only after reverse(k+2), its previous reader, ended.
    // Events: 0/1 recompute of an even/odd segment done, 2/3 reverse of an
    // even/odd segment done, 4 fork, 5 join.
    const hipStream_t s2 = b->rstream;
    hipEvent_t* ev = b->revents;
    rc = hip_check(hipEventRecord(ev[4], s), "hipEventRecord");
    if (!rc) rc = hip_check(hipStreamWaitEvent(s2, ev[4], 0), "hipStreamWaitEvent");
    if (rc) return rc;
    const int64_t last = L.n_ck - 1;
    rc = recompute(last, s2);
    if (!rc) rc = hip_check(hipEventRecord(ev[last % 2], s2), "hipEventRecord");
    for (int64_t k = last; k >= 0 && !rc; --k) {
      if (k >= 1) {
        // buffer (k-1) % 2 was last read by reverse(k+1)
        if (k + 1 <= last)
          rc = hip_check(hipStreamWaitEvent(s2, ev[2 + (k + 1) % 2], 0),
                         "hipStreamWaitEvent");
        if (!rc) rc = recompute(k - 1, s2);
        if (!rc)
          rc = hip_check(hipEventRecord(ev[(k - 1) % 2], s2), "hipEventRecord");
        if (rc) break;
      }
      rc = hip_check(hipStreamWaitEvent(s, ev[k % 2], 0), "hipStreamWaitEvent");
      if (!rc) rc = reverse(k);
      if (!rc) rc = hip_check(hipEventRecord(ev[2 + k % 2], s), "hipEventRecord");
    }
    // join the side stream even after a failure, so that a capture ends
    const int r1 = hip_check(hipEventRecord(ev[5], s2), "hipEventRecord");
    const int r2 = hip_check(hipStreamWaitEvent(s, ev[5], 0), "hipStreamWaitEvent");
    if (!rc) rc = r1 ? r1 : r2;
    if (rc) return rc;
  }
  if (cur != fbar &&
      (rc = hip_check(hipMemcpyAsync(fbar, cur, sizeof(double) * SD,
                                     hipMemcpyDeviceToDevice, s),
                      "hipMemcpyAsync")))
    return rc;
  hipLaunchKernelGGL(k_rbar_reduce, dim3((unsigned)((b->n_inst + 255) / 256)),
                     dim3(256), 0, s,
                     at<int64_t>(ws, b->adj_plain ? L.adj_first : L.rev_first),
                     b->n_inst, (const double*)slots, rbar);
  return hip_check(hipGetLastError(), "k_rbar_reduce");
}

lbm_batch* single_batch(lbm_handle* h) {
  if (h->one) return h->one;
  const int64_t offs[2] = {0, h->n};
  if (lbm_batch_init(&h->one, 1, offs, &h->p, h->stream) != LBM_OK) return nullptr;
  if (h->tune.kernel == LBM_KERNEL_BLOCKED) lbm_batch_set_tuning(h->one, &h->tune);
  return h->one;
}

// The handle's batch with the handle's current tile shape and reverse
// kernel: the workspace size and the checkpointed forward must see the same.
lbm_batch* synced_batch(lbm_handle* h) {
  lbm_batch* b = single_batch(h);
  if (!b) return nullptr;
  if (h->tune.kernel == LBM_KERNEL_BLOCKED && !same_tuning(b->tune, h->tune))
    lbm_batch_set_tuning(b, &h->tune);
  b->adj_kernel = h->adj_kernel;
  b->rec_stride = h->rec_stride;
  return b;
}

}  // namespace

namespace lbm {
void drop_adjoint_graph(lbm_batch* b) {
  if (b->adj_exec) (void)hipGraphExecDestroy(b->adj_exec);
  b->adj_exec = nullptr;
  b->ag_fbar = nullptr;
  b->ag_rbar = nullptr;
}
}  // namespace lbm

extern "C" {

size_t lbm_batch_adjoint_workspace_bytes(const lbm_batch* b, int64_t nsteps,
                                         int64_t ckpt_every) {
  if (!b || nsteps < 0 || ckpt_every < 1) return 0;
  return adj_layout(b, nsteps, ckpt_every,
                    current_plan(b)).total;
}

int lbm_batch_forward_ckpt(lbm_batch* b, double* f, void* ws, size_t ws_bytes,
                           int64_t nsteps, int64_t ckpt_every) {
  if (!b || !f || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (nsteps < 0 || ckpt_every < 1)
    return set_err(LBM_EINVAL, "need nsteps >= 0 and ckpt_every >= 1");
  // AUTO: the blocked reverse kernel (a prefetching K-step tile) wherever
  // its tiles can hold the forward halo, else the one-step kernel
  b->adj_plain = resolve_adj_plain(b);
  b->adj_every = resolve_every(b, b->adj_plain);
  const AdjPlan plan = resolved_plan(b);
  const AdjLayout L = adj_layout(b, nsteps, ckpt_every, plan);
  if (ws_bytes < L.total)
    return set_err(LBM_EWORKSPACE, "adjoint workspace of %zu bytes, need %zu",
                   ws_bytes, L.total);
  if (overlaps(f, sizeof(double) * 6 * b->n_total, ws, ws_bytes))
    return set_err(LBM_EINVAL, "f and ws overlap");
  if (((uintptr_t)f | (uintptr_t)ws) & 7)
    return set_err(LBM_EINVAL, "f and ws must be 8-byte aligned");
  if (!b->adj_plain && plan.rev.out() < 1)
    return set_err(LBM_ENOTSUP,
                   "the blocked adjoint kernel's tiles (P = 4, 8 wavefronts "
                   "for this shape) cannot hold a halo of 2K = %d nodes; use "
                   "the one-step adjoint kernel or a smaller K",
                   2 * b->tune.steps_per_launch);
  if (L.seg_bufs == 2) {
    // the pipelined reverse sweep's side stream (default priority) and
    // events, created once, outside any capture
    if (!b->rstream) {
      const int r = hip_check(
          hipStreamCreateWithFlags(&b->rstream, hipStreamNonBlocking),
          "hipStreamCreate");
      if (r) return r;
    }
    for (hipEvent_t& ev : b->revents)
      if (!ev) {
        const int r = hip_check(
            hipEventCreateWithFlags(&ev, hipEventDisableTiming),
            "hipEventCreate");
        if (r) return r;
      }
  }
  const hipStream_t s = b->stream;
  int rc = LBM_OK;
  const bool same = b->adj_ws == ws && b->adj_nsteps == nsteps &&
                    b->adj_ckpt == ckpt_every &&
                    same_tuning(b->adj_tune, b->tune) &&
                    b->adj_plain_up == b->adj_plain &&
                    b->adj_every_up == b->adj_every;
  if (!same) {
    // tables of this workspace layout: forward and recompute tiles (the
    // forward tile shape), tiles of the blocked and of the one-step reverse
    // kernels, and each lattice's first tile in the two reverse tables
    const lbm_tuning ft = fwd_tuning(b);
    const auto fwd = tile_table(b, tile_width(ft) - 4 * ft.steps_per_launch);
    const auto rec = tile_table(
        b, tile_width(rec_tuning(b->tune)) - 4 * b->tune.steps_per_launch);
    const auto rev = tile_table(b, plan.rev.out());
    const auto adj = tile_table(b, kAdjOut);
    auto firsts = [&](const std::vector<TileRef>& tab) {
      std::vector<int64_t> first(b->n_inst + 1, 0);
      for (const TileRef& t : tab) first[t.inst + 1]++;
      for (int64_t i = 0; i < b->n_inst; ++i) first[i + 1] += first[i];
      return first;
    };
    const auto first = firsts(adj);
    const auto rfirst = firsts(rev);
    auto up = [&](size_t off, const void* src, size_t bytes) {
      if (!rc && bytes)
        rc = hip_check(hipMemcpyAsync(at<char>(ws, off), src, bytes,
                                      hipMemcpyHostToDevice, s),
                       "hipMemcpyAsync");
    };
    up(L.consts, b->consts.data(), sizeof(Consts) * b->n_inst);
    up(L.offs, b->offsets.data(), sizeof(int64_t) * (b->n_inst + 1));
    up(L.fwd_tiles, fwd.data(), sizeof(TileRef) * fwd.size());
    up(L.rec_tiles, rec.data(), sizeof(TileRef) * rec.size());
    up(L.rev_tiles, rev.data(), sizeof(TileRef) * rev.size());
    up(L.adj_tiles, adj.data(), sizeof(TileRef) * adj.size());
    up(L.adj_first, first.data(), sizeof(int64_t) * first.size());
    up(L.rev_first, rfirst.data(), sizeof(int64_t) * rfirst.size());
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (rc) return rc;
    drop_adjoint_graph(b);
    b->adj_ws = ws;
    b->adj_nsteps = nsteps;
    b->adj_ckpt = ckpt_every;
    b->adj_tune = b->tune;
    b->adj_plain_up = b->adj_plain;
    b->adj_every_up = b->adj_every;
  }
  return enqueue_forward_ckpt(b, ws, f, nsteps, ckpt_every, L, s);
}

int lbm_batch_adjoint(lbm_batch* b, void* ws, size_t ws_bytes, int64_t nsteps,
                      int64_t ckpt_every, double* fbar, double* rbar,
                      int use_graph) {
  int rc = check_adj(b, ws, ws_bytes, nsteps, ckpt_every);
  if (rc) return rc;
  if (!fbar || !rbar) return set_err(LBM_EINVAL, "NULL argument");
  if (overlaps(fbar, sizeof(double) * 6 * b->n_total, ws, ws_bytes))
    return set_err(LBM_EINVAL, "fbar overlaps the workspace");
  if (!use_graph) return enqueue_adjoint(b, ws, nsteps, ckpt_every, fbar, rbar, b->stream);
  if (!(b->adj_exec && b->ag_fbar == fbar && b->ag_rbar == rbar)) {
    drop_adjoint_graph(b);
    if (!b->cap &&
        (rc = hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking),
                        "hipStreamCreate")))
      return rc;
    if ((rc = hip_check(hipStreamBeginCapture(b->cap,
                                              hipStreamCaptureModeThreadLocal),
                        "hipStreamBeginCapture")))
      return rc;
    const int rc_enq = enqueue_adjoint(b, ws, nsteps, ckpt_every, fbar, rbar, b->cap);
    hipGraph_t graph = nullptr;
    rc = hip_check(hipStreamEndCapture(b->cap, &graph), "hipStreamEndCapture");
    if (rc_enq) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc_enq;
    }
    if (rc) return rc;
    rc = hip_check(hipGraphInstantiate(&b->adj_exec, graph, nullptr, nullptr, 0),
                   "hipGraphInstantiate");
    (void)hipGraphDestroy(graph);
    if (rc) {
      b->adj_exec = nullptr;
      return rc;
    }
    b->ag_fbar = fbar;
    b->ag_rbar = rbar;
  }
  return hip_check(hipGraphLaunch(b->adj_exec, b->stream), "hipGraphLaunch");
}

int lbm_batch_loss(lbm_batch* b, const double* f, const double* target,
                   void* ws, size_t ws_bytes, double* loss, double* fbar) {
  if (!b || !f || !ws || !loss || !fbar) return set_err(LBM_EINVAL, "NULL argument");
  if (b->adj_ws != ws || ws_bytes < adj_layout(b, b->adj_nsteps, b->adj_ckpt, resolved_plan(b)).total)
    return set_err(LBM_EINVAL, "call lbm_batch_forward_ckpt with this workspace first");
  const AdjLayout L = adj_layout(b, b->adj_nsteps, b->adj_ckpt, resolved_plan(b));
  hipLaunchKernelGGL(k_loss, dim3((unsigned)b->n_inst), dim3(256), 0, b->stream,
                     at<Consts>(ws, L.consts), at<int64_t>(ws, L.offs), f, target,
                     loss, fbar, b->n_total);
  return hip_check(hipGetLastError(), "k_loss");
}

int lbm_batch_equilibrium_adjoint(lbm_batch* b, const double* rho,
                                  const double* J, const double* zeta,
                                  const double* fbar, double* rho_bar,
                                  double* J_bar, double* zeta_bar, void* ws,
                                  size_t ws_bytes) {
  if (!b || !rho || !J || !zeta || !fbar || !rho_bar || !J_bar || !zeta_bar || !ws)
    return set_err(LBM_EINVAL, "NULL argument");
  if (b->adj_ws != ws || ws_bytes < adj_layout(b, b->adj_nsteps, b->adj_ckpt, resolved_plan(b)).total)
    return set_err(LBM_EINVAL, "call lbm_batch_forward_ckpt with this workspace first");
  const AdjLayout L = adj_layout(b, b->adj_nsteps, b->adj_ckpt, resolved_plan(b));
  hipLaunchKernelGGL(k_equilibrium_adjoint, dim3((unsigned)b->n_inst), dim3(256),
                     0, b->stream, at<Consts>(ws, L.consts),
                     at<int64_t>(ws, L.offs), rho, J, zeta, fbar, rho_bar,
                     J_bar, zeta_bar, b->n_total);
  return hip_check(hipGetLastError(), "k_equilibrium_adjoint");
}

int lbm_batch_moments_adjoint(lbm_batch* b, const double* mbar, double* fbar,
                              void* ws, size_t ws_bytes) {
  if (!b || !mbar || !fbar || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (b->adj_ws != ws || ws_bytes < adj_layout(b, b->adj_nsteps, b->adj_ckpt, resolved_plan(b)).total)
    return set_err(LBM_EINVAL, "call lbm_batch_forward_ckpt with this workspace first");
  const AdjLayout L = adj_layout(b, b->adj_nsteps, b->adj_ckpt, resolved_plan(b));
  hipLaunchKernelGGL(k_moments_adjoint, dim3((unsigned)b->n_inst), dim3(256), 0,
                     b->stream, at<Consts>(ws, L.consts), at<int64_t>(ws, L.offs),
                     mbar, fbar, b->n_total);
  return hip_check(hipGetLastError(), "k_moments_adjoint");
}

int lbm_batch_set_adjoint_kernel(lbm_batch* b, int kernel) {
  if (!b) return set_err(LBM_EINVAL, "batch is NULL");
  if (kernel != LBM_KERNEL_AUTO && kernel != LBM_KERNEL_PLAIN &&
      kernel != LBM_KERNEL_BLOCKED)
    return set_err(LBM_EINVAL, "unknown adjoint kernel %d", kernel);
  b->adj_kernel = kernel;
  return LBM_OK;
}

// ----------------------------------------------------- single lattice --

int lbm_batch_set_recompute_stride(lbm_batch* b, int stride) {
  if (!b) return set_err(LBM_EINVAL, "batch is NULL");
  if (stride < 0 || stride > 2)
    return set_err(LBM_EINVAL, "recompute stride must be 0, 1 or 2, not %d",
                   stride);
  b->rec_stride = stride;
  return LBM_OK;
}
int lbm_set_recompute_stride(lbm_handle* h, int stride) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  if (stride < 0 || stride > 2)
    return set_err(LBM_EINVAL, "recompute stride must be 0, 1 or 2, not %d",
                   stride);
  h->rec_stride = stride;
  return LBM_OK;
}
int lbm_set_adjoint_kernel(lbm_handle* h, int kernel) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  if (kernel != LBM_KERNEL_AUTO && kernel != LBM_KERNEL_PLAIN &&
      kernel != LBM_KERNEL_BLOCKED)
    return set_err(LBM_EINVAL, "unknown adjoint kernel %d", kernel);
  h->adj_kernel = kernel;
  return LBM_OK;
}

size_t lbm_adjoint_workspace_bytes(lbm_handle* h, int64_t nsteps,
                                   int64_t ckpt_every) {
  if (!h) return 0;
  lbm_batch* b = synced_batch(h);
  // rbar staging for the host copy lives in the scratch region
  return b ? lbm_batch_adjoint_workspace_bytes(b, nsteps, ckpt_every) : 0;
}

int lbm_forward_ckpt(lbm_handle* h, double* f, void* ws, size_t ws_bytes,
                     int64_t nsteps, int64_t ckpt_every) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  lbm_batch* b = synced_batch(h);
  if (!b) return LBM_EINVAL;
  return lbm_batch_forward_ckpt(b, f, ws, ws_bytes, nsteps, ckpt_every);
}

int lbm_adjoint(lbm_handle* h, void* ws, size_t ws_bytes, int64_t nsteps,
                int64_t ckpt_every, double* fbar, double rbar[3], int use_graph) {
  if (!h || !rbar) return set_err(LBM_EINVAL, "NULL argument");
  lbm_batch* b = single_batch(h);
  if (!b) return LBM_EINVAL;
  const AdjLayout L = adj_layout(b, nsteps, ckpt_every, resolved_plan(b));
  double* dev = at<double>(ws, L.scratch);
  int rc = lbm_batch_adjoint(b, ws, ws_bytes, nsteps, ckpt_every, fbar, dev,
                             use_graph);
  if (!rc)
    rc = hip_check(hipMemcpyAsync(rbar, dev, 3 * sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream),
                   "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return rc;
}

int lbm_loss(lbm_handle* h, const double* f, const double* target, void* ws,
             size_t ws_bytes, double* loss, double* fbar) {
  if (!h || !loss) return set_err(LBM_EINVAL, "NULL argument");
  lbm_batch* b = single_batch(h);
  if (!b) return LBM_EINVAL;
  if (b->adj_ws != ws) return set_err(LBM_EINVAL, "call lbm_forward_ckpt first");
  const AdjLayout L = adj_layout(b, b->adj_nsteps, b->adj_ckpt, resolved_plan(b));
  double* dev = at<double>(ws, L.scratch);
  int rc = lbm_batch_loss(b, f, target, ws, ws_bytes, dev, fbar);
  if (!rc)
    rc = hip_check(hipMemcpyAsync(loss, dev, sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream),
                   "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return rc;
}

int lbm_equilibrium_adjoint(lbm_handle* h, const double* rho, const double* J,
                            const double* zeta, const double* fbar,
                            double* rho_bar, double* J_bar, double* zeta_bar,
                            void* ws, size_t ws_bytes) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  lbm_batch* b = single_batch(h);
  if (!b) return LBM_EINVAL;
  return lbm_batch_equilibrium_adjoint(b, rho, J, zeta, fbar, rho_bar, J_bar,
                                       zeta_bar, ws, ws_bytes);
}

int lbm_moments_adjoint(lbm_handle* h, const double* mbar, double* fbar,
                        void* ws, size_t ws_bytes) {
  if (!h) return set_err(LBM_EINVAL, "handle is NULL");
  lbm_batch* b = single_batch(h);
  if (!b) return LBM_EINVAL;
  return lbm_batch_moments_adjoint(b, mbar, fbar, ws, ws_bytes);
}

}  // extern "C"
