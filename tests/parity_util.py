"""Shared helpers of the parity tests: parameter sets given identically to the
oracle and to the GPU library, the per-field error metric, and seeded states."""
import numpy as np

import oracle

# Per-field relative error: max |gpu - oracle| over a field divided by
# max(|oracle field|_inf, 1e-3 |whole state|_inf); the floor keeps fields
# that vanish at rest (g for s0 = 0) from dividing by ~0.
FLOOR = 1e-3
TOL = 1e-12

PARAM_SETS = {
    "paper": dict(),
    "odd": dict(lam=1.7, cp=2.3, rho0=1.3, gamma=1.31, prandtl=0.71, c0=0.61,
                s0=0.37, s_e=1.37, s_eps=1.1),
    "nosource": dict(s_e=1.6, source_on=0),
    "linear": dict(eq_kind=1, u0_lin=0.15, s0_lin=0.2, s_e=1.9),
    "fluid": dict(eq_kind=2, source_on=0, s_e=1.7, c0=0.55),
    "thermal": dict(eq_kind=3, source_on=0, u0_lin=0.2, alpha=-0.5, s_e=1.6,
                    s_psi=1.3),
    # the single-distribution schemes away from unit scales (lambda, rho0,
    # cp != 1), where the device's scaled moments differ from the physical
    "fluid_odd": dict(eq_kind=2, source_on=0, s_e=1.5, lam=1.3, rho0=1.2,
                      cp=1.7, c0=0.7, gamma=1.3),
    "thermal_odd": dict(eq_kind=3, source_on=0, u0_lin=0.25, alpha=0.3,
                        s_e=1.4, s_psi=1.2, lam=1.4, rho0=0.9, cp=2.1, c0=0.6),
}


def oracle_params(name: str, **kw) -> oracle.Params:
    d = dict(PARAM_SETS[name])
    d.update(kw)
    p = oracle.Params(**d)
    if p.s_psi is None:
        p.s_psi = oracle.coupled_rates(p.s_e, p.gamma, p.prandtl)[0]
    return p


def gpu_params(po: oracle.Params):
    from paper_1802_02369_amd import lbm
    return lbm.Params(lam=po.lam, rho0=po.rho0, cp=po.cp, gamma=po.gamma,
                      prandtl=po.prandtl, c0=po.c0, s0=po.s0, s_e=po.s_e,
                      s_psi=po.s_psi, s_eps=po.s_eps, u0_lin=po.u0_lin,
                      s0_lin=po.s0_lin, alpha=po.alpha, source_on=po.source_on,
                      eq_kind=po.eq_kind)


def field_errors(got: np.ndarray, want: np.ndarray) -> np.ndarray:
    scale = np.abs(want).max()
    den = np.maximum(np.abs(want).max(axis=-1), FLOOR * scale)
    return np.abs(got - want).max(axis=-1) / den


def max_err(got, want) -> float:
    return float(field_errors(got, want).max())


def random_fields(rng, n, p: oracle.Params, amp=0.2, u=0.1, ds=0.3):
    rho = p.rho0 * (1 + amp * rng.uniform(-1, 1, n))
    J = rho * u * p.lam * rng.uniform(-1, 1, n)
    zeta = rho * (p.s0 + ds * p.cp * rng.uniform(-1, 1, n))
    return rho, J, zeta


def random_state(rng, n, p: oracle.Params, **kw):
    """A seeded non-equilibrium state (equilibrium times 1 +- 1e-3 noise)."""
    f = oracle.init(*random_fields(rng, n, p, **kw), p)
    return f * (1 + 1e-3 * rng.uniform(-1, 1, f.shape))


def window_oracle(fields, j: int, k: int, p: oracle.Params) -> np.ndarray:
    """Oracle value of node j of a periodic lattice after k steps, from the
    2k-node neighbourhood that determines it (one step has radius 2): the
    window of 4k + 3 nodes around j is run as its own periodic lattice, whose
    wrap-around cannot reach the centre within k steps."""
    rho, J, zeta = fields
    n = len(rho)
    idx = (j + np.arange(-2 * k - 1, 2 * k + 2)) % n
    f = oracle.init(rho[idx], J[idx], zeta[idx], p)
    f = oracle.run(f, k, p)
    return f[:, 2 * k + 1]
