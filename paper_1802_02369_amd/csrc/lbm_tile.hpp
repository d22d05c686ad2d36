// Register-tile helpers shared by the forward and reverse tile kernels:
// coalesced loads and stores of a wavefront's segment through LDS, and the
// per-step boundary record exchanged between the wavefronts of a tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace {

// Global memory is touched only at the start and the end of the launch, and
// always coalesced: node i of a wavefront's segment travels through that
// wavefront's LDS buffer between the coalesced order (lane l handles
// i = k*64 + l) and the register order (lane l owns i = l*P + k).  The LDS
// index i + i/P pads one double per lane row so that both orders are free of
// bank conflicts.  Staging is private to a wavefront (wave_barrier only).
template <int P>
__device__ __forceinline__ int lds_idx(int i) {
  return i + i / P;
}

__device__ __forceinline__ int64_t wrap_near(int64_t x, int64_t n, bool small) {
  if (small) return lbm::wrap_mod(x, n);
  return x < 0 ? x + n : (x >= n ? x - n : x);
}

// Arrays of a lattice of length L are at fin + q*S (S >= L, the array
// stride of the state the lattice lives in).
template <int P>
__device__ __forceinline__ void tile_load(const double* __restrict__ fin,
                                          int64_t S, int64_t n, int64_t start,
                                          bool inside, bool small, int lane,
                                          double* lds, double (&f)[6][P]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double* src = fin + (int64_t)q * S;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int i = k * 64 + lane;
      const int64_t g = inside ? start + i : wrap_near(start + i, n, small);
      lds[lds_idx<P>(i)] = src[g];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < P; ++k) f[q][k] = lds[lds_idx<P>(lane * P + k)];
    __builtin_amdgcn_wave_barrier();
  }
}

// tile_load in three parts, for a kernel that reloads the same segment of
// successive states: the global indices of the coalesced order (computed
// once), the global loads into registers in that order (which may be issued
// a step ahead), and the pass through LDS into the register order.
template <int P>
__device__ __forceinline__ void tile_index(int64_t n, int64_t start,
                                           bool inside, bool small, int lane,
                                           int64_t (&gi)[P]) {
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int i = k * 64 + lane;
    gi[k] = inside ? start + i : wrap_near(start + i, n, small);
  }
}

template <int P>
__device__ __forceinline__ void tile_fetch(const double* __restrict__ fin,
                                           int64_t S, const int64_t (&gi)[P],
                                           double (&raw)[6][P]) {
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int k = 0; k < P; ++k) raw[q][k] = fin[(int64_t)q * S + gi[k]];
}

template <int P>
__device__ __forceinline__ void tile_transpose(int lane, double* lds,
                                               const double (&raw)[6][P],
                                               double (&f)[6][P]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) {
#pragma unroll
    for (int k = 0; k < P; ++k) lds[lds_idx<P>(k * 64 + lane)] = raw[q][k];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < P; ++k) f[q][k] = lds[lds_idx<P>(lane * P + k)];
    __builtin_amdgcn_wave_barrier();
  }
}

// Stores the nodes of this wavefront's segment whose tile index lies in
// [lo, hi) and whose global index is below n.
template <int P>
__device__ __forceinline__ void tile_store(double* __restrict__ fout,
                                           int64_t S, int64_t n, int64_t start,
                                           int lo, int hi, int lane, double* lds,
                                           const double (&f)[6][P]) {
  // one 64-bit lane base and a wavefront-uniform upper bound keep few
  // values live around a kernel's step loop
  const int64_t g0 = start + lane;
  const int64_t lim = n - start;  // i < lim  <=>  start + i < n
#pragma unroll
  for (int q = 0; q < 6; ++q) {
#pragma unroll
    for (int k = 0; k < P; ++k) lds[lds_idx<P>(lane * P + k)] = f[q][k];
    __builtin_amdgcn_wave_barrier();
    double* dst = fout + (int64_t)q * S + g0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int i = k * 64 + lane;
      if (i >= lo && i < hi && i < lim) dst[k * 64] = lds[lds_idx<P>(i)];
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// One time step of a wavefront's nodes.  The source of node k needs u, T of
// k-1 and k+1, so the collisions run in the order P-1, 0, 1, ..., P-2 and
// each source is applied as soon as its right neighbour exists; only a window
// of three nodes' (u, T) stays live besides the populations.
// SAVE: also keeps each node's thermodynamic state of the incoming state in
// th[k] (the reverse sweep reuses it for that state's own reverse step).
template <int P, int EQ, bool SAVE = false>
__device__ __forceinline__ void tile_step(const lbm::Consts& c, double (&f)[6][P],
                                          lbm::NodeThermo* th = nullptr) {
  if constexpr (P == 1) {
    // one node per lane: both neighbours are the adjacent lanes
    double u, T, rw, w;
    lbm::collide_local<EQ, SAVE>(c, f[0][0], f[1][0], f[2][0], f[3][0], f[4][0],
                                 f[5][0], u, T, rw, w, th);
    const double add =
        lbm::source_g(c, rw, w, lbm::from_left(u), lbm::from_right(u),
                      lbm::from_left(T), lbm::from_right(T));
    f[3][0] += add;
    f[4][0] += add;
    f[5][0] += add;
    f[1][0] = lbm::from_left(f[1][0]);
    f[4][0] = lbm::from_left(f[4][0]);
    f[2][0] = lbm::from_right(f[2][0]);
    f[5][0] = lbm::from_right(f[5][0]);
    return;
  }
  double uA, TA, rwA, wA;  // node P-1, collided first
  lbm::collide_local<EQ, SAVE>(c, f[0][P - 1], f[1][P - 1], f[2][P - 1],
                               f[3][P - 1], f[4][P - 1], f[5][P - 1], uA, TA,
                               rwA, wA, SAVE ? th + (P - 1) : nullptr);
  double um, Tm, rwm, wm;  // node k (the one whose source is next)
  __builtin_amdgcn_sched_barrier(0);
  lbm::collide_local<EQ, SAVE>(c, f[0][0], f[1][0], f[2][0], f[3][0], f[4][0],
                               f[5][0], um, Tm, rwm, wm, th);
  double ul = lbm::from_left(uA), Tl = lbm::from_left(TA);
  const double uR = lbm::from_right(um), TR = lbm::from_right(Tm);
#pragma unroll
  for (int k = 0; k < P; ++k) {
    double ur, Tr, rwr = 0.0, wr = 0.0;
    // Keep the scheduler from interleaving the collisions of different
    // nodes: that would hold several nodes' temporaries live at once.
    __builtin_amdgcn_sched_barrier(0);
    if (k + 1 < P - 1) {
      lbm::collide_local<EQ, SAVE>(c, f[0][k + 1], f[1][k + 1], f[2][k + 1],
                                   f[3][k + 1], f[4][k + 1], f[5][k + 1], ur, Tr,
                                   rwr, wr, SAVE ? th + (k + 1) : nullptr);
    } else if (k + 1 == P - 1) {
      ur = uA;
      Tr = TA;
      rwr = rwA;
      wr = wA;
    } else {
      ur = uR;
      Tr = TR;
    }
    const double add = lbm::source_g(c, rwm, wm, ul, ur, Tl, Tr);
    f[3][k] += add;
    f[4][k] += add;
    f[5][k] += add;
    ul = um;
    Tl = Tm;
    um = ur;
    Tm = Tr;
    rwm = rwr;
    wm = wr;
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

// Values exchanged between neighbouring wavefronts of a workgroup each step.
struct Boundary {
  double v[8];
};

}  // namespace
