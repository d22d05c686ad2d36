"""Seeded synthetic workloads (initial fields and per-lattice rates).

The paper's experiments (section 9) are periodic acoustic waves; there is no
dataset.  These generators produce the initial density, momentum and volumic
entropy fields (rho, J, zeta = rho s) and the relaxation rate s_e of each
lattice, on the host as numpy arrays, from numpy ``default_rng(seed)``.  They
hold no arithmetic of the scheme itself: the equilibrium populations, the
coupled rates s_psi(s_e) and everything after are computed separately by the
GPU library and by the test oracle from these same arrays.

Gas constants for every workload follow section 9: gamma = 1.4, Pr = 1,
c0 = lambda / 2, s0 = 0, with lambda = rho0 = cp = 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAMMA, PRANDTL, C0, CP, RHO0, S0, LAM = 1.4, 1.0, 0.5, 1.0, 1.0, 0.0, 1.0

# Largest relaxation rate s_e for which the linearised coupled scheme stays
# stable about every local state of a standing sine wave of the given
# amplitude (frozen-coefficient Fourier analysis; the scheme is stable for all
# s_e in (0, 2) at rest and loses stability at high wavenumber about moving
# states).  Columns: amplitude, ceiling.
STANDING_CEILING = np.array([
    [0.00, 2.000], [0.01, 2.000], [0.05, 1.987], [0.10, 1.943],
    [0.15, 1.861], [0.20, 1.720], [0.30, 1.106]])


def standing_ceiling(a: np.ndarray) -> np.ndarray:
    return np.interp(a, STANDING_CEILING[:, 0], STANDING_CEILING[:, 1])


@dataclass
class Fields:
    rho: np.ndarray
    J: np.ndarray
    zeta: np.ndarray


@dataclass
class Batch:
    offsets: np.ndarray   # int64 [n_inst + 1]
    s_e: np.ndarray       # float64 [n_inst]
    amp: np.ndarray       # float64 [n_inst]
    fields: Fields        # concatenated over instances

    @property
    def n_inst(self) -> int:
        return len(self.offsets) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def instance(self, i: int) -> Fields:
        a, b = self.offsets[i], self.offsets[i + 1]
        return Fields(self.fields.rho[a:b], self.fields.J[a:b],
                      self.fields.zeta[a:b])


def uniform_temperature_wave(n: int, amp: float, seed: int) -> Fields:
    """Rest state plus a density sine of one wavelength over the lattice with
    a seeded phase, at rest (u = 0) and uniform temperature, i.e. specific
    entropy s = s0 - ((gamma - 1)/gamma) cp ln(rho/rho0) (eq. gaz-parfait at
    constant T)."""
    rng = np.random.default_rng(seed)
    phi = 2 * np.pi * rng.uniform()
    j = np.arange(n)
    rho = RHO0 * (1 + amp * np.sin(2 * np.pi * j / n + phi))
    s = S0 - (GAMMA - 1) / GAMMA * CP * np.log(rho / RHO0)
    return Fields(rho, np.zeros(n), rho * s)


def progressive_wave(n: int, amp: float, wavelength: int, seed: int) -> Fields:
    """Right-going acoustic wave: rho = rho0 (1 + a sin(2 pi j / wavelength
    + phi)), u = c0 (rho - rho0)/rho0, s = s0 (isentropic)."""
    rng = np.random.default_rng(seed)
    phi = 2 * np.pi * rng.uniform()
    j = np.arange(n)
    rho = RHO0 * (1 + amp * np.sin(2 * np.pi * j / wavelength + phi))
    u = C0 * (rho - RHO0) / RHO0
    return Fields(rho, rho * u, rho * S0)


def multimode(n: int, modes: int, amp: float, seed: int) -> Fields:
    """rho = rho0 + sum_m amp sin(2 pi m j / n + phi_m), J = sum_m amp c0
    sin(2 pi m j / n + phi'_m), zeta = 0, m = 1..modes, seeded phases."""
    rng = np.random.default_rng(seed)
    phi = 2 * np.pi * rng.uniform(size=modes)
    psi = 2 * np.pi * rng.uniform(size=modes)
    j = np.arange(n)
    rho = np.full(n, RHO0)
    J = np.zeros(n)
    for m in range(1, modes + 1):
        rho += amp * np.sin(2 * np.pi * m * j / n + phi[m - 1])
        J += amp * C0 * np.sin(2 * np.pi * m * j / n + psi[m - 1])
    return Fields(rho, J, np.zeros(n))


def standing_batch(lengths: np.ndarray, amps: np.ndarray, s_e: np.ndarray,
                   rng: np.random.Generator) -> Batch:
    """Standing one-wavelength density sines (u = 0, s = s0) on each lattice."""
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    rho = np.empty(offsets[-1])
    phases = 2 * np.pi * rng.uniform(size=len(lengths))
    for i, L in enumerate(lengths):
        j = np.arange(L)
        rho[offsets[i]:offsets[i + 1]] = RHO0 * (
            1 + amps[i] * np.sin(2 * np.pi * j / L + phases[i]))
    return Batch(offsets, s_e.astype(np.float64), amps.astype(np.float64),
                 Fields(rho, np.zeros_like(rho), rho * S0))


# ------------------------------------------------------------ configs -----

def config_small(seed: int = 0):
    """N = 256, amplitude 1e-3 at uniform temperature, s_e = 1.9, 1000 steps."""
    return dict(n=256, steps=1000, s_e=1.9,
                fields=uniform_temperature_wave(256, 1e-3, seed))


def config_large(n: int = 1 << 24, seed: int = 1, steps: int = 2000):
    """Single lattice, progressive wave of amplitude 0.2 and wavelength 128
    nodes (so that it steepens into shocks within the run), s_e = 0.9."""
    return dict(n=n, steps=steps, s_e=0.9,
                fields=progressive_wave(n, 0.2, 128, seed))


def config_batched(n_inst: int = 4096, seed: int = 2, steps: int = 5000,
                   lmin: int = 512, lmax: int = 16384):
    """Lengths log-uniform in [lmin, lmax], amplitudes U[1e-3, 0.3], s_e
    uniform in [0.5, ceiling(a) - 0.05] capped at 1.95."""
    rng = np.random.default_rng(seed)
    L = np.rint(np.exp(rng.uniform(np.log(lmin), np.log(lmax), n_inst))).astype(np.int64)
    a = rng.uniform(1e-3, 0.3, n_inst)
    hi = np.minimum(standing_ceiling(a) - 0.05, 1.95)
    s_e = rng.uniform(0.5, hi)
    b = standing_batch(L, a, s_e, rng)
    return dict(batch=b, steps=steps)


def config_adjoint(n: int = 8192, steps: int = 10000, ckpt: int = 100):
    """Eight-mode initial field (seed 3), target from the same construction
    with seed 4 run for the same number of steps, s_e = 1.9."""
    return dict(n=n, steps=steps, ckpt=ckpt, s_e=1.9,
                fields=multimode(n, 8, 0.01, 3),
                target_fields=multimode(n, 8, 0.01, 4))


def config_batched_adjoint(n_inst: int = 1024, seed: int = 5, steps: int = 4000,
                           ckpt: int = 63, lmin: int = 1024, lmax: int = 8192):
    """Lengths uniform in [lmin, lmax], amplitudes U[0.01, 0.2], s_e uniform
    in [0.5, min(1.9, ceiling(a) - 0.05)]; loss 1/2 sum (rho(T) - rho0)^2."""
    rng = np.random.default_rng(seed)
    L = rng.integers(lmin, lmax + 1, n_inst).astype(np.int64)
    a = rng.uniform(0.01, 0.2, n_inst)
    hi = np.minimum(standing_ceiling(a) - 0.05, 1.9)
    s_e = rng.uniform(0.5, hi)
    b = standing_batch(L, a, s_e, rng)
    return dict(batch=b, steps=steps, ckpt=ckpt)
