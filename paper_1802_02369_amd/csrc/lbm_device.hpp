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
  int32_t eq_kind;  // 0 section 8, 1 linear, 2 isentropic fluid D1Q3
  int32_t pad;
};

// One tile of a batched launch: tile t of lattice inst.
struct TileRef {
  int32_t inst;
  int32_t t;
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

// Thermodynamics from conserved moments: u, T and w = 1/T, plus X = ln(T/T0).
__device__ __forceinline__ void thermo(const Consts& c, double rho, double J,
                                       double zeta, double& u, double& s,
                                       double& X, double& T) {
  const double ir = 1.0 / rho;
  u = J * ir;
  s = zeta * ir;
  X = c.gm1 * log(rho * c.irho0) + (c.gcp * s + c.xs0);
  T = c.T0 * exp(X);
}

// Isentropic pressure p0 (rho/rho0)^gamma = rho r T0 (rho/rho0)^(gamma-1)
// of the fluid D1Q3 scheme (sections 2-3).
__device__ __forceinline__ double iso_pressure(const Consts& c, double rho) {
  return rho * c.r * c.T0 * exp(c.gm1 * log(rho * c.irho0));
}

// Steps (ii)-(vi) at one node, in place on the six populations: moments,
// equilibria, relaxation, back to populations.  Returns u, T and the two
// factors the source needs: rw = rho / T and w = 1 / T.
__device__ __forceinline__ void collide_local(const Consts& c, double& f0,
                                              double& fp, double& fm,
                                              double& g0, double& gp,
                                              double& gm, double& u, double& T,
                                              double& rw, double& w) {
  // (ii) moments, eq. M-d1q3q3
  const double sf = fp + fm;
  const double rho = density(c, f0, fp, fm);
  const double J = c.mJ * (fp - fm);
  const double e = c.me * (sf - 2.0 * f0);
  const double sg = gp + gm;
  const double zeta = c.mz * (g0 + sg);
  const double psi = c.mpsi * (gp - gm);
  const double eps = c.meps * (sg - 2.0 * g0);
  // (iv) equilibria
  double s, X;
  thermo(c, rho, J, zeta, u, s, X, T);
  double e_eq, psi_eq, eps_eq;
  if (c.eq_kind == 0) {
    const double p = rho * c.r * T;
    e_eq = 3.0 * (J * u + p) - c.two_l2 * rho;
    psi_eq = zeta * u;
    eps_eq = c.eps_c * rho * X + e_eq * s;
  } else if (c.eq_kind == 2) {
    e_eq = 3.0 * (J * u + iso_pressure(c, rho)) - c.two_l2 * rho;
    psi_eq = 0.0;
    eps_eq = 0.0;
  } else {
    e_eq = c.lin[0] * rho + c.lin[1] * J + c.lin[2] * zeta;
    psi_eq = c.lin[3] * rho + c.lin[4] * J + c.lin[5] * zeta;
    eps_eq = c.lin[6] * rho + c.lin[7] * J + c.lin[8] * zeta;
  }
  // (v) relaxation, eq. relaxation-d1q3q3
  const double es = e + c.s_e * (e_eq - e);
  const double psis = psi + c.s_psi * (psi_eq - psi);
  const double epss = eps + c.s_eps * (eps_eq - eps);
  // (vi) f* = M^-1 m*
  const double fr = c.fa * rho, fe = c.fb * es, fj = c.fc * J;
  f0 = fr - fe;
  fp = fr + 0.5 * fe + fj;
  fm = fr + 0.5 * fe - fj;
  const double gz = c.ga * zeta, ge = c.gb * epss, gj = c.gc * psis;
  g0 = gz - ge;
  gp = gz + 0.5 * ge + gj;
  gm = gz + 0.5 * ge - gj;
  w = 1.0 / T;
  rw = rho * w;
}

// u and T of a node (used for the halo nodes of the one-step kernel).
__device__ __forceinline__ void node_uT(const Consts& c, double f0, double fp,
                                        double fm, double g0, double gp,
                                        double gm, double& u, double& T) {
  const double rho = density(c, f0, fp, fm);
  const double J = c.mJ * (fp - fm);
  const double zeta = c.mz * (g0 + (gp + gm));
  double s, X;
  thermo(c, rho, J, zeta, u, s, X, T);
}

// Step (vii): the increment of zeta at node j, already divided into the
// M^-1 column of zeta (each of g0, g+, g- receives ga * dz).
__device__ __forceinline__ double source_g(const Consts& c, double rw, double w,
                                           double uL, double uR, double TL,
                                           double TR) {
  const double du = uR - uL;
  const double dT = TR - TL;
  const double dz = c.src_c * rw * (du * du + c.cPr * (dT * dT) * w);
  return c.ga * dz;
}

// Equilibrium populations from (rho, J, zeta).
__device__ __forceinline__ void equilibrium(const Consts& c, double rho,
                                            double J, double zeta, double f[6]) {
  double u, s, X, T;
  thermo(c, rho, J, zeta, u, s, X, T);
  double e_eq, psi_eq, eps_eq;
  if (c.eq_kind == 0) {
    const double p = rho * c.r * T;
    e_eq = 3.0 * (J * u + p) - c.two_l2 * rho;
    psi_eq = zeta * u;
    eps_eq = c.eps_c * rho * X + e_eq * s;
  } else if (c.eq_kind == 2) {
    e_eq = 3.0 * (J * u + iso_pressure(c, rho)) - c.two_l2 * rho;
    psi_eq = 0.0;
    eps_eq = 0.0;
  } else {
    e_eq = c.lin[0] * rho + c.lin[1] * J + c.lin[2] * zeta;
    psi_eq = c.lin[3] * rho + c.lin[4] * J + c.lin[5] * zeta;
    eps_eq = c.lin[6] * rho + c.lin[7] * J + c.lin[8] * zeta;
  }
  const double fr = c.fa * rho, fe = c.fb * e_eq, fj = c.fc * J;
  f[0] = fr - fe;
  f[1] = fr + 0.5 * fe + fj;
  f[2] = fr + 0.5 * fe - fj;
  const double gz = c.ga * zeta, ge = c.gb * eps_eq, gj = c.gc * psi_eq;
  f[3] = gz - ge;
  f[4] = gz + 0.5 * ge + gj;
  f[5] = gz + 0.5 * ge - gj;
}

// Cross-lane moves of a double over the whole 64-lane wavefront (DPP
// wave_shr:1 / wave_shl:1 on both 32-bit halves).  from_left: lane l receives
// lane l-1's value; from_right: lane l receives lane l+1's value.  The edge
// lane (0, resp. 63) keeps its own value.
__device__ __forceinline__ double from_left(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi2, lo2);
}
__device__ __forceinline__ double from_right(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ int64_t wrap_mod(int64_t x, int64_t n) {
  int64_t r = x % n;
  return r < 0 ? r + n : r;
}

}  // namespace lbm
