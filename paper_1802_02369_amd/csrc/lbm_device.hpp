// Device-side arithmetic of one node of the coupled D1Q3Q3 scheme
// (Dubois, Graille & Lallemand, arXiv 1802.02369, section 8, steps (ii)-(vii)).
//
// Formulation used on the GPU (algebraically equal to the paper's, fewer
// transcendental calls):
//   X = ln(T/T0) = (gamma-1) ln(rho/rho0) + gamma (s - s0)/cp, T = T0 e^X,
//   p = rho r T with r = cp (gamma-1)/gamma.  This is eq. gaz-parfait with
//   T0 = p0 / (rho0 r), p0 = rho0 c0^2 / gamma: one log and one exp per node.
//   eps_eq = (2 cp lambda^2 / gamma) rho X + e_eq s, because the bracket of
//   eq. eq-energie-entropie-d1q3q3 equals e_eq of eq. energie-equilibre.
//   Step (vii): dt S_j = (sigma_e/4) (rho_j/T_j) [(u_{j+1}-u_{j-1})^2
//   + (cp/Pr) (T_{j+1}-T_{j-1})^2 / T_j], from S of eq. NS-rho-J-zeta with
//   centred differences, nu = sigma_e lambda dx (eq. nu-d1q3q3),
//   kappa = rho nu cp / Pr and dt = dx / lambda: dx cancels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Per-lattice constants derived on the host from lbm_params.
struct Consts {
  double rho0, irho0;
  double mJ, me;      // rho0 lambda, rho0 lambda^2
  double mz, mpsi, meps;  // rho0 cp, rho0 cp lambda, rho0 cp lambda^2
  double gm1, gcp, xs0;   // gamma - 1, gamma / cp, -gamma s0 / cp
  double T0, r;
  double two_l2;      // 2 lambda^2
  double eps_c;       // 2 cp lambda^2 / gamma
  double s_e, s_psi, s_eps;
  double src_c;       // sigma_e / 4, or 0 without the source
  double cPr;         // cp / Pr
  double fa, fb, fc;  // M^-1 for f: 1/(3 rho0), 1/(3 rho0 lambda^2), 1/(2 rho0 lambda)
  double ga, gb, gc;  // M^-1 for g: same with rho0 cp
  double gamma, cp;
  // linear equilibria (section 7, and the thermal scheme of section 4):
  // e = l[0] rho + l[1] J + l[2] zeta, psi = l[3..5] . W, eps = l[6..8] . W
  double lin[9];
  double xs0l;         // xs0 - (gamma - 1) ln rho0
  // The time step in scaled moments (see collide_local):
  double se_2, se_3, se_6;  // s_e / 2, s_e / 3, s_e / 6
  double ise2;              // 1 / s_e^2 (d sigma_e / d s_e = -1 / s_e^2)
  double sp_2, sx_3, sx_6;  // s_psi / 2, s_eps / 3, s_eps / 6
  double hP;                // c0^2 / (gamma lambda^2) = p0 / (rho0 lambda^2)
  double two_g;             // 2 / gamma
  double hS, hC;            // source: src_c lambda^2 / (3 cp T0), cp T0 / (Pr lambda^2)
  double hSd;               // d hS / d s_e = -lambda^2 / (12 cp T0 s_e^2), or 0
  double hlin[9];           // linear equilibria in scaled moments
  int32_t eq_kind;  // 0 section 8, 1 linear, 2 isentropic fluid D1Q3
  int32_t flags;    // lbm_params.flags (LBM_CHECK_FINITE)
};

// One tile of a batched launch: tile t of lattice inst.
struct TileRef {
  int32_t inst;
  int32_t t;
};

// A lattice of a batch held in one workgroup's registers for a whole run
// (see k_batch_resident): wavefronts wave0 .. wave0 + nw - 1 of its
// workgroup.
struct ResidentItem {
  int32_t inst;
  int32_t wave0;
  int32_t nw;
  int32_t pad;
};

// rho = rho0 f0 + rho0 f+ + rho0 f-, summed in the order of the first row of
// eq. M-d1q3q3 without contraction.  X contains (gamma-1) ln rho, so a one-ulp
// change of rho moves eps_eq by ~1e-16 in absolute terms; a fixed order keeps
// rho reproducible across implementations.
__device__ __forceinline__ double density(const Consts& c, double f0, double fp,
                                          double fm) {
#pragma clang fp contract(off)
  const double a = c.rho0 * f0;
  const double b = c.rho0 * fp;
  const double d = c.rho0 * fm;
  return (a + b) + d;
}

// 1/x for the positive normal numbers of the step (rho, T): the hardware
// reciprocal estimate r (relative error e = 1 - x r below 2^-22) refined by
// one third-order step r (1 + e + e^2) = (1 - e^3)/x, within one ulp of 1/x
// (not always correctly rounded).
__device__ __forceinline__ double recip(double x) {
#pragma clang fp contract(off)
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// ln 2 = kLn2Hi + kLn2Lo: kLn2Hi is ln 2 rounded to 42 significant bits, so
// that n kLn2Hi is exact for |n| < 2^11; kLn2Lo is the rest rounded to double.
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
constexpr double kLog2e = 0x1.71547652b82fep+0;     // 1 / ln 2
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;  // sqrt(1/2)

// Natural logarithm of a positive finite x.  Method: x = m 2^k with m in
// [sqrt(1/2), sqrt(2)); ln m = 2 atanh(z) with z = (m-1)/(m+1), |z| < 0.172,
// written z (2 + w Q(w)), w = z^2, where Q is a degree-6 Chebyshev fit of
// (2 atanh(z) - 2z)/z^3 on [0, 0.02944] (relative error of the fit below
// 5e-18; coefficients from csrc/gen_poly.py); ln x = k ln 2 + ln m with ln 2
// in two parts (the additive reduction of Cody & Waite).  Error a few ulp.
// x <= 0 gives NaN; so do NaN and +inf.
//
// ln_reduce splits x: the hardware mantissa mh in [1/2, 1) and a = 2 when
// mh < sqrt(1/2), else 1, so that m = a mh exactly; m - 1 and m + 1 are
// then single FMAs (a mh - 1 is exact).  ln_finish completes ln x from z.
struct LnReduced {
  double mh, a;
  int k;
};

__device__ __forceinline__ LnReduced ln_reduce(double x) {
  LnReduced r;
  r.mh = __builtin_amdgcn_frexp_mant(x);
  const bool lo = r.mh < kSqrtHalf;
  r.a = lo ? 2.0 : 1.0;
  r.k = __builtin_amdgcn_frexp_exp(x) - (lo ? 1 : 0);
  return r;
}

__device__ __forceinline__ double ln_finish(double x, const LnReduced& rd,
                                            double z) {
#pragma clang fp contract(off)
  const double w = z * z;
  double q = 0x1.2b584c80de001p-3;
  q = fma(q, w, 0x1.39fe603f8739ep-3);
  q = fma(q, w, 0x1.7462b4ac51915p-3);
  q = fma(q, w, 0x1.c71c62e57c0cfp-3);
  q = fma(q, w, 0x1.2492492df14bfp-2);
  q = fma(q, w, 0x1.99999999952e2p-2);
  q = fma(q, w, 0x1.5555555555558p-1);
  const double lm = z * fma(w, q, 2.0);
  const double kd = (double)rd.k;
  const double r = fma(kd, kLn2Hi, fma(kd, kLn2Lo, lm));
  // x <= 0: replace the high word by a quiet-NaN pattern (one select)
  const uint64_t b = __builtin_bit_cast(uint64_t, r);
  const uint32_t hi = x > 0.0 ? (uint32_t)(b >> 32) : 0x7ff80000u;
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (b & 0xffffffffu));
}

__device__ __forceinline__ double ln_pos(double x) {
#pragma clang fp contract(off)
  const LnReduced rd = ln_reduce(x);
  const double z = fma(rd.a, rd.mh, -1.0) * recip(fma(rd.a, rd.mh, 1.0));
  return ln_finish(x, rd, z);
}

// ln x and 1/x of a positive finite x with one reciprocal: R = 1/(x (m+1))
// gives 1/x = R (m+1) and 1/(m+1) = R x (each within about two ulp: the
// rounding of x (m+1), of R and of the product).  Non-positive, NaN or
// infinite x give a NaN logarithm, as ln_pos.
__device__ __forceinline__ double ln_inv(double x, double& inv) {
#pragma clang fp contract(off)
  const LnReduced rd = ln_reduce(x);
  const double d = fma(rd.a, rd.mh, 1.0);
  const double R = recip(x * d);
  inv = R * d;
  const double z = fma(rd.a, rd.mh, -1.0) * (R * x);
  return ln_finish(x, rd, z);
}

// e^x for the moderate arguments of the equation of state.  Method (Cody &
// Waite): n = nearest integer to x / ln 2, r = x - n ln 2 with ln 2 in two
// parts, |r| <= 0.3466; e^r = 1 + r (1 + r R(r)) where R is a degree-9
// Chebyshev fit of (e^r - 1 - r)/r^2 (relative error of e^r below 2e-17;
// coefficients from csrc/gen_poly.py); e^x = 2^n e^r.  Error a few ulp.
// Overflow gives +inf and underflow 0 (the hardware saturates n); NaN stays
// NaN.
__device__ __forceinline__ double exp_fin(double x) {
#pragma clang fp contract(off)
  const double n = __builtin_rint(x * kLog2e);
  const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, x));
  double q = 0x1.af38a71a18cb9p-26;
  q = fma(q, r, 0x1.2891834686c7ep-22);
  q = fma(q, r, 0x1.71de0daf7a6ccp-19);
  q = fma(q, r, 0x1.a019b90eefe8ep-16);
  q = fma(q, r, 0x1.a01a01a7c3d59p-13);
  q = fma(q, r, 0x1.6c16c1788b646p-10);
  q = fma(q, r, 0x1.11111111109b4p-7);
  q = fma(q, r, 0x1.5555555553d64p-5);
  q = fma(q, r, 0x1.5555555555556p-3);
  q = fma(q, r, 0x1.0000000000001p-1);
  q = fma(q, r, 1.0);
  q = fma(q, r, 1.0);
  return __builtin_amdgcn_ldexp(q, (int)n);
}

// Every function below fixes its own rounding sequence: contraction of a
// product and a sum into an FMA is off, and FMAs are written where wanted.
// A node-update therefore rounds identically in every kernel that inlines
// these functions (one-step, any tile shape, batched), and those kernels
// produce bitwise identical states.

// Thermodynamics from conserved moments: u, s and X = ln(T/T0), T; ir
// returns 1/rho.
__device__ __forceinline__ void thermo(const Consts& c, double rho, double J,
                                       double zeta, double& u, double& s,
                                       double& X, double& T, double& ir) {
#pragma clang fp contract(off)
  const double lr = ln_inv(rho, ir);
  u = J * ir;
  s = zeta * ir;
  X = fma(c.gm1, lr, fma(c.gcp, s, c.xs0l));
  T = c.T0 * exp_fin(X);
}

__device__ __forceinline__ void thermo(const Consts& c, double rho, double J,
                                       double zeta, double& u, double& s,
                                       double& X, double& T) {
  double ir;
  thermo(c, rho, J, zeta, u, s, X, T, ir);
}

// Isentropic pressure p0 (rho/rho0)^gamma = rho r T0 (rho/rho0)^(gamma-1)
// of the fluid D1Q3 scheme (sections 2-3).
__device__ __forceinline__ double iso_pressure(const Consts& c, double rho) {
#pragma clang fp contract(off)
  return ((rho * c.r) * c.T0) * exp_fin(c.gm1 * ln_pos(rho * c.irho0));
}

// Step (iv): equilibria of the non-conserved moments from rho, J, zeta and
// the thermodynamic state (physical units; the initialisation uses them).
template <int EQ>
__device__ __forceinline__ void equilibria(const Consts& c, double rho,
                                           double J, double zeta, double u,
                                           double s, double X, double T,
                                           double& e_eq, double& psi_eq,
                                           double& eps_eq) {
#pragma clang fp contract(off)
  if (EQ == 0 || c.eq_kind == 0) {
    e_eq = fma(3.0, fma(J, u, (rho * c.r) * T), -(c.two_l2 * rho));
    psi_eq = zeta * u;
    eps_eq = fma(e_eq, s, (c.eps_c * rho) * X);
  } else if (c.eq_kind == 2) {
    e_eq = fma(3.0, fma(J, u, iso_pressure(c, rho)), -(c.two_l2 * rho));
    psi_eq = 0.0;
    eps_eq = 0.0;
  } else {
    e_eq = fma(c.lin[2], zeta, fma(c.lin[1], J, c.lin[0] * rho));
    psi_eq = fma(c.lin[5], zeta, fma(c.lin[4], J, c.lin[3] * rho));
    eps_eq = fma(c.lin[8], zeta, fma(c.lin[7], J, c.lin[6] * rho));
  }
}

// The time step works in scaled moments, which removes the scale factors
// rho0, lambda, cp, T0 from the per-node arithmetic:
//   rh = rho/rho0 = f0 + f+ + f-,  Jh = J/(rho0 lambda) = f+ - f-,
//   zh = zeta/(rho0 cp) = g0 + g+ + g-,  uh = u/lambda,  sh = s/cp,
//   Th = T/T0 = e^X,  X = (gamma-1) ln rh + gamma sh - gamma s0/cp,
// and the equilibria divided by the scale of their moment (rho0 lambda^2 for
// e, rho0 cp lambda for psi, rho0 cp lambda^2 for eps):
//   eh = 3 (Jh uh + hP rh Th) - 2 rh,  psih = zh uh,
//   epsh = (2/gamma) rh X + eh sh,  hP = c0^2/(gamma lambda^2).
// (With rho0 = 1, rh is the density summed in the order of eq. M-d1q3q3.)
// lr returns ln rh.
// ir returns 1/rh.
__device__ __forceinline__ void thermo_scaled(const Consts& c, double rh,
                                              double Jh, double zh, double& uh,
                                              double& sh, double& X,
                                              double& Th, double& lr,
                                              double& ir) {
#pragma clang fp contract(off)
  lr = ln_inv(rh, ir);
  uh = Jh * ir;
  sh = zh * ir;
  X = fma(c.gm1, lr, fma(c.gamma, sh, c.xs0));
  Th = exp_fin(X);
}

__device__ __forceinline__ void thermo_scaled(const Consts& c, double rh,
                                              double Jh, double zh, double& uh,
                                              double& sh, double& X,
                                              double& Th, double& lr) {
  double ir;
  thermo_scaled(c, rh, Jh, zh, uh, sh, X, Th, lr, ir);
}

// The thermodynamic state of a node's incoming populations, as the time
// step computes it (kept by the reverse sweep for a state it recomputes).
struct NodeThermo {
  double uh, sh, X, Th, lr, ir, w;
};

// Steps (ii)-(vi) at one node, in place on the six populations: moments,
// equilibria, relaxation, back to populations.  Returns uh, Th and the two
// factors the source needs: rw = rh / Th and w = 1 / Th.  EQ = 0 compiles
// the equilibria of section 8 only (every lattice of the launch has
// eq_kind 0); EQ = -1 selects them per lattice from c.eq_kind.  SAVE: also
// writes the node's thermodynamic state into *save.
template <int EQ, bool SAVE = false>
__device__ __forceinline__ void collide_local(const Consts& c, double& f0,
                                              double& fp, double& fm,
                                              double& g0, double& gp,
                                              double& gm, double& u, double& T,
                                              double& rw, double& w,
                                              NodeThermo* save = nullptr) {
#pragma clang fp contract(off)
  // (ii) the conserved moments, eq. M-d1q3q3, scaled
  const double rh = (f0 + fp) + fm;
  const double Jh = fp - fm;
  const double sg = gp + gm;
  const double zh = g0 + sg;
  // (iv) equilibria
  double sh, X, lr, ir;
  thermo_scaled(c, rh, Jh, zh, u, sh, X, T, lr, ir);
  double jup, eh, psih, epsh;
  if (EQ == 0 || c.eq_kind == 0) {
    jup = fma(Jh, u, (c.hP * rh) * T);
    eh = fma(-2.0, rh, 3.0 * jup);
    psih = zh * u;
    epsh = fma(eh, sh, (c.two_g * rh) * X);
  } else if (c.eq_kind == 2) {
    jup = fma(Jh, u, (c.hP * rh) * exp_fin(c.gm1 * lr));
    eh = fma(-2.0, rh, 3.0 * jup);
    psih = 0.0;
    epsh = 0.0;
  } else {
    jup = 0.0;
    eh = fma(c.hlin[2], zh, fma(c.hlin[1], Jh, c.hlin[0] * rh));
    psih = fma(c.hlin[5], zh, fma(c.hlin[4], Jh, c.hlin[3] * rh));
    epsh = fma(c.hlin[8], zh, fma(c.hlin[7], Jh, c.hlin[6] * rh));
  }
  // (v) relaxation (eq. relaxation-d1q3q3) and (vi) f* = M^-1 m*, combined:
  // only e, psi, eps change, so f* = f + M^-1 (m* - m).  The entries of M^-1
  // turn the changes into
  //   de = fb (e* - e) = (s_e/3) (eh - (f+ + f- - 2 f0)),
  //   dp = gc (psi* - psi) = (s_psi/2) (psih - (g+ - g-)),
  //   dx = gb (eps* - eps) = (s_eps/3) (epsh - (g+ + g- - 2 g0)),
  // and f0 -= de, f+- += de/2; g0 -= dx, g+- += dx/2 +- dp.  When
  // eh = 3 (Jh uh + hP rh Th) - 2 rh, de reduces to
  // s_e (Jh uh + hP rh Th - (f+ + f-)) since rh = f0 + f+ + f-.  The rates
  // enter through the FMAs of the updates.
  if (EQ == 0 || c.eq_kind != 1) {
    const double d = jup - (fp + fm);
    f0 = fma(-c.s_e, d, f0);
    fp = fma(c.se_2, d, fp);
    fm = fma(c.se_2, d, fm);
  } else {
    const double d = eh - fma(-2.0, f0, fp + fm);
    f0 = fma(-c.se_3, d, f0);
    fp = fma(c.se_6, d, fp);
    fm = fma(c.se_6, d, fm);
  }
  const double dpr = psih - (gp - gm);
  const double dxr = epsh - fma(-2.0, g0, sg);
  g0 = fma(-c.sx_3, dxr, g0);
  gp = fma(c.sp_2, dpr, fma(c.sx_6, dxr, gp));
  gm = fma(-c.sp_2, dpr, fma(c.sx_6, dxr, gm));
  w = recip(T);
  rw = rh * w;
  if constexpr (SAVE) *save = NodeThermo{u, sh, X, T, lr, ir, w};
}

// uh and Th of a node (the halo nodes of the one-step kernel), rounded as in
// collide_local.
__device__ __forceinline__ void node_uT(const Consts& c, double f0, double fp,
                                        double fm, double g0, double gp,
                                        double gm, double& u, double& T) {
#pragma clang fp contract(off)
  const double rh = (f0 + fp) + fm;
  const double Jh = fp - fm;
  const double zh = g0 + (gp + gm);
  double sh, X, lr;
  thermo_scaled(c, rh, Jh, zh, u, sh, X, T, lr);
}

// Step (vii): the increment of zeta at node j, already divided into the
// M^-1 column of zeta (each of g0, g+, g- receives ga dt S_j), from scaled
// quantities: ga dt S_j = hS rh wh [(uh_{j+1} - uh_{j-1})^2
// + hC (Th_{j+1} - Th_{j-1})^2 wh] with wh = 1/Th_j.
__device__ __forceinline__ double source_g(const Consts& c, double rw, double w,
                                           double uL, double uR, double TL,
                                           double TR) {
#pragma clang fp contract(off)
  const double du = uR - uL;
  const double dT = TR - TL;
  return (c.hS * rw) * fma(du, du, (c.hC * (dT * dT)) * w);
}

// Equilibrium populations from (rho, J, zeta).
__device__ __forceinline__ void equilibrium(const Consts& c, double rho,
                                            double J, double zeta, double f[6]) {
#pragma clang fp contract(off)
  double u, s, X, T;
  thermo(c, rho, J, zeta, u, s, X, T);
  double e_eq, psi_eq, eps_eq;
  equilibria<-1>(c, rho, J, zeta, u, s, X, T, e_eq, psi_eq, eps_eq);
  const double fr = c.fa * rho, fe = c.fb * e_eq, fj = c.fc * J;
  f[0] = fr - fe;
  f[1] = fma(0.5, fe, fr) + fj;
  f[2] = fma(0.5, fe, fr) - fj;
  const double gz = c.ga * zeta, ge = c.gb * eps_eq, gj = c.gc * psi_eq;
  f[3] = gz - ge;
  f[4] = fma(0.5, ge, gz) + gj;
  f[5] = fma(0.5, ge, gz) - gj;
}

// Cross-lane moves of a double over the whole 64-lane wavefront (DPP
// wave_shr:1 / wave_shl:1 on both 32-bit halves).  from_left: lane l receives
// lane l-1's value; from_right: lane l receives lane l+1's value.  The edge
// lane (0, resp. 63) has no source and receives 0 (bound_ctrl); callers use
// it only for nodes whose values are discarded or replaced.
__device__ __forceinline__ double from_left(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t wrap_mod(int64_t x, int64_t n) {
  int64_t r = x % n;
  return r < 0 ? r + n : r;
}

}  // namespace lbm
