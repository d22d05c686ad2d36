"""Reference oracle of the coupled D1Q3Q3 lattice Boltzmann scheme.

TEST INFRASTRUCTURE ONLY.  A plain single-threaded FP64 C++ implementation
(``lbm_oracle.cpp``) written from the paper (Dubois, Graille & Lallemand,
arXiv 1802.02369, sections 2-8), reached through ctypes.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package; the
GPU library never does.

State layout: numpy float64 array of shape (6, n) holding f0, f+, f-, g0, g+,
g- (the particle vector f_d of section 6) on a periodic lattice of n nodes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with g++."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", *CXXFLAGS, _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("lam", ctypes.c_double), ("rho0", ctypes.c_double),
        ("cp", ctypes.c_double), ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double), ("c0", ctypes.c_double),
        ("s0", ctypes.c_double), ("dx", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_psi", ctypes.c_double),
        ("s_eps", ctypes.c_double),
        ("u0_lin", ctypes.c_double), ("s0_lin", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("source_on", ctypes.c_int32), ("eq_kind", ctypes.c_int32),
    ]


@dataclass
class Params:
    """Physical and lattice constants of one lattice (section 9 defaults)."""
    lam: float = 1.0
    rho0: float = 1.0
    cp: float = 1.0
    gamma: float = 1.4
    prandtl: float = 1.0
    c0: float = 0.5
    s0: float = 0.0
    dx: float = 1.0
    s_e: float = 1.9
    s_psi: float | None = None   # None: coupled to s_e (section 7)
    s_eps: float = 1.5
    u0_lin: float = 0.0
    s0_lin: float = 0.0
    alpha: float = 0.0
    source_on: int = 1
    eq_kind: int = 0

    def c(self) -> OrcParams:
        s_psi = self.s_psi
        if s_psi is None:
            s_psi, _ = coupled_rates(self.s_e, self.gamma, self.prandtl)
        return OrcParams(self.lam, self.rho0, self.cp, self.gamma,
                         self.prandtl, self.c0, self.s0, self.dx, self.s_e,
                         s_psi, self.s_eps, self.u0_lin, self.s0_lin,
                         self.alpha, int(self.source_on), int(self.eq_kind))

    def rates(self) -> tuple[float, float, float]:
        p = self.c()
        return p.s_e, p.s_psi, p.s_eps


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_P = ctypes.POINTER(OrcParams)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        sig = {
            "orc_coupled_rates": [ctypes.c_double] * 3 + [_D, _D],
            "orc_rate_from_viscosity": [ctypes.c_double] * 3 + [_D],
            "orc_moment_matrix": [_P, _D, _D],
            "orc_moments": [_I64, _D, _P, _D],
            "orc_equilibria": [_I64, _D, _D, _D, _P, _D],
            "orc_source": [_I64, _D, _P, _D],
            "orc_init": [_I64, _D, _D, _D, _P, _D],
            "orc_step": [_I64, _D, _P, _D],
            "orc_run": [_I64, _D, _I64, _P],
            "orc_diagnostics": [_I64, _D, _P, _D],
            "orc_step_tlm": [_I64, _D, _D, _D, _P, _D, _D],
            "orc_step_adjoint": [_I64, _D, _D, _P, _D, _D],
            "orc_init_tlm": [_I64, _D, _D, _D, _D, _D, _D, _P, _D, _D],
            "orc_init_adjoint": [_I64, _D, _D, _D, _D, _P, _D, _D, _D],
            "orc_loss": [_I64, _D, _D, _P, _D, _D],
            "orc_gradient": [_I64, _D, _D, _D, _I64, _I64, _D, _P, _D, _D,
                             _D, _D, _D],
            "orc_directional": [_I64, _D, _D, _D, _D, _D, _D, _D, _I64, _D,
                                _P, _D, _D],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _check(rc: int, name: str):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments (rc={rc})")


def coupled_rates(s_e: float, gamma: float = 1.4, prandtl: float = 1.0):
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().orc_coupled_rates(s_e, gamma, prandtl, ctypes.byref(a),
                                   ctypes.byref(b)), "coupled_rates")
    return a.value, b.value


def rate_from_viscosity(nu: float, lam: float, dx: float) -> float:
    a = ctypes.c_double()
    _check(lib().orc_rate_from_viscosity(nu, lam, dx, ctypes.byref(a)),
           "rate_from_viscosity")
    return a.value


def moment_matrix(p: Params):
    M = np.zeros((6, 6))
    Mi = np.zeros((6, 6))
    cp = p.c()
    _check(lib().orc_moment_matrix(ctypes.byref(cp), _ptr(M), _ptr(Mi)),
           "moment_matrix")
    return M, Mi


def moments(f, p: Params) -> np.ndarray:
    f = _arr(f)
    n = f.shape[-1]
    m = np.zeros((6, n))
    cp = p.c()
    _check(lib().orc_moments(n, _ptr(f), ctypes.byref(cp), _ptr(m)), "moments")
    return m


def equilibria(rho, J, zeta, p: Params) -> np.ndarray:
    """Rows: e_eq, psi_eq, eps_eq, p, T."""
    rho, J, zeta = _arr(rho), _arr(J), _arr(zeta)
    n = rho.shape[0]
    out = np.zeros((5, n))
    cp = p.c()
    _check(lib().orc_equilibria(n, _ptr(rho), _ptr(J), _ptr(zeta),
                                ctypes.byref(cp), _ptr(out)), "equilibria")
    return out


def source(f, p: Params) -> np.ndarray:
    f = _arr(f)
    n = f.shape[-1]
    out = np.zeros(n)
    cp = p.c()
    _check(lib().orc_source(n, _ptr(f), ctypes.byref(cp), _ptr(out)), "source")
    return out


def init(rho, J, zeta, p: Params) -> np.ndarray:
    rho, J, zeta = _arr(rho), _arr(J), _arr(zeta)
    n = rho.shape[0]
    f = np.zeros((6, n))
    cp = p.c()
    _check(lib().orc_init(n, _ptr(rho), _ptr(J), _ptr(zeta), ctypes.byref(cp),
                          _ptr(f)), "init")
    return f


def step(f, p: Params) -> np.ndarray:
    f = _arr(f)
    out = np.zeros_like(f)
    cp = p.c()
    _check(lib().orc_step(f.shape[-1], _ptr(f), ctypes.byref(cp), _ptr(out)),
           "step")
    return out


def run(f, nsteps: int, p: Params) -> np.ndarray:
    f = _arr(f).copy()
    cp = p.c()
    _check(lib().orc_run(f.shape[-1], _ptr(f), int(nsteps), ctypes.byref(cp)),
           "run")
    return f


def diagnostics(f, p: Params) -> np.ndarray:
    f = _arr(f)
    out = np.zeros(8)
    cp = p.c()
    _check(lib().orc_diagnostics(f.shape[-1], _ptr(f), ctypes.byref(cp),
                                 _ptr(out)), "diagnostics")
    return out


def step_tlm(f, df, dr, p: Params):
    f, df, dr = _arr(f), _arr(df), _arr(dr)
    fo, dfo = np.zeros_like(f), np.zeros_like(f)
    cp = p.c()
    _check(lib().orc_step_tlm(f.shape[-1], _ptr(f), _ptr(df), _ptr(dr),
                              ctypes.byref(cp), _ptr(fo), _ptr(dfo)),
           "step_tlm")
    return fo, dfo


def step_adjoint(f, fbar_next, p: Params):
    f, fb = _arr(f), _arr(fbar_next)
    out = np.zeros_like(f)
    rbar = np.zeros(3)
    cp = p.c()
    _check(lib().orc_step_adjoint(f.shape[-1], _ptr(f), _ptr(fb),
                                  ctypes.byref(cp), _ptr(out), _ptr(rbar)),
           "step_adjoint")
    return out, rbar


def init_tlm(rho, J, zeta, drho, dJ, dzeta, p: Params):
    a = [_arr(x) for x in (rho, J, zeta, drho, dJ, dzeta)]
    n = a[0].shape[0]
    f, df = np.zeros((6, n)), np.zeros((6, n))
    cp = p.c()
    _check(lib().orc_init_tlm(n, *[_ptr(x) for x in a], ctypes.byref(cp),
                              _ptr(f), _ptr(df)), "init_tlm")
    return f, df


def init_adjoint(rho, J, zeta, fbar, p: Params):
    rho, J, zeta, fbar = _arr(rho), _arr(J), _arr(zeta), _arr(fbar)
    n = rho.shape[0]
    out = [np.zeros(n) for _ in range(3)]
    cp = p.c()
    _check(lib().orc_init_adjoint(n, _ptr(rho), _ptr(J), _ptr(zeta),
                                  _ptr(fbar), ctypes.byref(cp),
                                  *[_ptr(x) for x in out]), "init_adjoint")
    return tuple(out)


def loss(f, target, p: Params):
    f, target = _arr(f), _arr(target)
    fbar = np.zeros_like(f)
    L = ctypes.c_double()
    cp = p.c()
    _check(lib().orc_loss(f.shape[-1], _ptr(f), _ptr(target), ctypes.byref(cp),
                          ctypes.byref(L), _ptr(fbar)), "loss")
    return L.value, fbar


def gradient(rho, J, zeta, nsteps: int, target, p: Params, ckpt: int = 0):
    """Returns (loss, rho_bar, J_bar, zeta_bar, rbar[3])."""
    rho, J, zeta, target = _arr(rho), _arr(J), _arr(zeta), _arr(target)
    n = rho.shape[0]
    out = [np.zeros(n) for _ in range(3)]
    rbar = np.zeros(3)
    L = ctypes.c_double()
    cp = p.c()
    _check(lib().orc_gradient(n, _ptr(rho), _ptr(J), _ptr(zeta), int(nsteps),
                              int(ckpt), _ptr(target), ctypes.byref(cp),
                              ctypes.byref(L), *[_ptr(x) for x in out],
                              _ptr(rbar)), "gradient")
    return L.value, out[0], out[1], out[2], rbar


def directional(rho, J, zeta, drho, dJ, dzeta, dr, nsteps: int, target,
                p: Params):
    """Returns (loss, dloss) for the direction (drho, dJ, dzeta, dr)."""
    a = [_arr(x) for x in (rho, J, zeta, drho, dJ, dzeta, dr)]
    target = _arr(target)
    n = a[0].shape[0]
    L, dL = ctypes.c_double(), ctypes.c_double()
    cp = p.c()
    _check(lib().orc_directional(n, *[_ptr(x) for x in a], int(nsteps),
                                 _ptr(target), ctypes.byref(cp),
                                 ctypes.byref(L), ctypes.byref(dL)),
           "directional")
    return L.value, dL.value
