"""Thin ctypes binding of ``liblbm.so`` (C ABI declared in include/lbm.h).

Argument marshalling only: every step of the scheme runs in the library's HIP
kernels.  Device memory comes from torch tensors (float64, CUDA/HIP device);
calls enqueue on torch's current stream.  If the built library is missing the
import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_EWORKSPACE, LBM_ENONFINITE, LBM_ENOTSUP = \
    0, -1, -2, -3, -4, -5
LBM_EUNSTABLE = -6
LBM_CHECK_FINITE = 1  # bit of Params.flags
KERNEL_AUTO, KERNEL_PLAIN, KERNEL_BLOCKED = 0, 1, 2
MAX_GROUPS = 4
RESIDENT_MIN, RESIDENT_MAX = 16, 5952  # lattice lengths of resident runs
NOALLOC_MAX_NODES = 1 << 20
WS_STEP, WS_TUNE = 0, 1


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class CParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in (
        "lam", "rho0", "cp", "gamma", "prandtl", "c0", "s0",
        "s_e", "s_psi", "s_eps", "u0_lin", "s0_lin", "alpha")] + [
        ("source_on", ctypes.c_int32), ("eq_kind", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CTuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("nodes_per_lane", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "lbm_last_error": ([], ctypes.c_char_p),
            "lbm_coupled_rates": ([_d, _d, _d, _dp, _dp, _dp], ctypes.c_int),
            "lbm_linear_stability": ([ctypes.POINTER(CParams), _d, _d, _d,
                                      ctypes.c_int32, _dp], ctypes.c_int),
            "lbm_init": ([ctypes.POINTER(_vp), _i64, ctypes.POINTER(CParams), _vp],
                         ctypes.c_int),
            "lbm_destroy": ([_vp], None),
            "lbm_set_stream": ([_vp, _vp], ctypes.c_int),
            "lbm_set_params": ([_vp, ctypes.POINTER(CParams)], ctypes.c_int),
            "lbm_workspace_bytes": ([_vp, ctypes.c_int], _sz),
            "lbm_set_tuning": ([_vp, ctypes.POINTER(CTuning)], ctypes.c_int),
            "lbm_get_tuning": ([_vp, ctypes.POINTER(CTuning)], ctypes.c_int),
            "lbm_set_equilibrium": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
            "lbm_step": ([_vp, _vp, _vp, _sz, _i64], ctypes.c_int),
            "lbm_step_noalloc": ([_vp, _vp, _i64], ctypes.c_int),
            "lbm_moments": ([_vp, _vp, _vp], ctypes.c_int),
            "lbm_diagnostics": ([_vp, _vp, _vp, _sz, _dp], ctypes.c_int),
            "lbm_autotune": ([_vp, _vp, _vp, _sz, _i64, ctypes.c_char_p,
                              ctypes.POINTER(CTuning)], ctypes.c_int),
            "lbm_batch_init": ([ctypes.POINTER(_vp), _i64,
                                ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(CParams), _vp], ctypes.c_int),
            "lbm_batch_destroy": ([_vp], None),
            "lbm_batch_set_stream": ([_vp, _vp], ctypes.c_int),
            "lbm_batch_set_tuning": ([_vp, ctypes.POINTER(CTuning)], ctypes.c_int),
            "lbm_batch_get_tuning": ([_vp, ctypes.POINTER(CTuning)], ctypes.c_int),
            "lbm_batch_set_groups": ([_vp, ctypes.c_int32, ctypes.POINTER(CTuning),
                                      ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "lbm_batch_get_groups": ([_vp, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(CTuning),
                                      ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "lbm_batch_total_nodes": ([_vp], _i64),
            "lbm_batch_set_resident": ([_vp, ctypes.c_int], ctypes.c_int),
            "lbm_batch_resident_lattices": ([_vp], _i64),
            "lbm_batch_workspace_bytes": ([_vp, ctypes.c_int], _sz),
            "lbm_batch_prepare": ([_vp, _vp, _sz], ctypes.c_int),
            "lbm_batch_set_equilibrium": ([_vp, _vp, _vp, _vp, _vp, _vp, _sz],
                                          ctypes.c_int),
            "lbm_batch_run": ([_vp, _vp, _vp, _sz, _i64, ctypes.c_int],
                              ctypes.c_int),
            "lbm_batch_diagnostics": ([_vp, _vp, _vp, _sz, _dp], ctypes.c_int),
            "lbm_batch_moments": ([_vp, _vp, _vp, _vp, _sz], ctypes.c_int),
            "lbm_batch_autotune": ([_vp, _vp, _vp, _sz, _i64, ctypes.c_char_p,
                                    ctypes.POINTER(CTuning)], ctypes.c_int),
            "lbm_adjoint_workspace_bytes": ([_vp, _i64, _i64], _sz),
            "lbm_forward_ckpt": ([_vp, _vp, _vp, _sz, _i64, _i64], ctypes.c_int),
            "lbm_adjoint": ([_vp, _vp, _sz, _i64, _i64, _vp, _dp, ctypes.c_int],
                            ctypes.c_int),
            "lbm_loss": ([_vp, _vp, _vp, _vp, _sz, _dp, _vp], ctypes.c_int),
            "lbm_equilibrium_adjoint": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _vp, _sz], ctypes.c_int),
            "lbm_moments_adjoint": ([_vp, _vp, _vp, _vp, _sz], ctypes.c_int),
            "lbm_batch_adjoint_workspace_bytes": ([_vp, _i64, _i64], _sz),
            "lbm_batch_forward_ckpt": ([_vp, _vp, _vp, _sz, _i64, _i64],
                                       ctypes.c_int),
            "lbm_batch_adjoint": ([_vp, _vp, _sz, _i64, _i64, _vp, _vp,
                                   ctypes.c_int], ctypes.c_int),
            "lbm_batch_loss": ([_vp, _vp, _vp, _vp, _sz, _vp, _vp], ctypes.c_int),
            "lbm_batch_equilibrium_adjoint": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                               _vp, _vp, _sz], ctypes.c_int),
            "lbm_batch_moments_adjoint": ([_vp, _vp, _vp, _vp, _sz],
                                          ctypes.c_int),
            "lbm_set_adjoint_kernel": ([_vp, ctypes.c_int], ctypes.c_int),
            "lbm_batch_set_adjoint_kernel": ([_vp, ctypes.c_int], ctypes.c_int),
            "lbm_set_recompute_stride": ([_vp, ctypes.c_int], ctypes.c_int),
            "lbm_batch_set_recompute_stride": ([_vp, ctypes.c_int], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int):
    if rc != LBM_OK:
        msg = lib().lbm_last_error().decode()
        raise LBMError(rc, msg)


def coupled_rates(s_e: float, gamma: float = 1.4, prandtl: float = 1.0):
    """(s_psi, s_eps, d s_psi / d s_e) of the section-7 coupling."""
    a, b, c = _d(), _d(), _d()
    check(lib().lbm_coupled_rates(s_e, gamma, prandtl, ctypes.byref(a),
                                  ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def linear_stability(p: "Params", rho: float = 1.0, u: float = 0.0,
                     s: float | None = None, nk: int = 256):
    """(max amplification, stable) of one step about the uniform state
    (rho, u, s) over nk Fourier modes in [0, pi] (lbm_linear_stability;
    s defaults to p.s0)."""
    a = _d()
    cp = p.c()
    rc = lib().lbm_linear_stability(ctypes.byref(cp), float(rho), float(u),
                                    float(p.s0 if s is None else s), int(nk),
                                    ctypes.byref(a))
    if rc not in (LBM_OK, LBM_EUNSTABLE):
        check(rc)
    return a.value, rc == LBM_OK


@dataclass
class Params:
    lam: float = 1.0
    rho0: float = 1.0
    cp: float = 1.0
    gamma: float = 1.4
    prandtl: float = 1.0
    c0: float = 0.5
    s0: float = 0.0
    s_e: float = 1.9
    s_psi: float | None = None  # None: coupled to s_e
    s_eps: float = 1.5
    u0_lin: float = 0.0
    s0_lin: float = 0.0
    alpha: float = 0.0
    source_on: int = 1
    eq_kind: int = 0
    flags: int = 0  # LBM_CHECK_FINITE: check every launch's output

    def c(self) -> CParams:
        s_psi = self.s_psi
        if s_psi is None:
            s_psi = coupled_rates(self.s_e, self.gamma, self.prandtl)[0]
        return CParams(self.lam, self.rho0, self.cp, self.gamma, self.prandtl,
                       self.c0, self.s0, self.s_e, s_psi, self.s_eps,
                       self.u0_lin, self.s0_lin, self.alpha,
                       int(self.source_on), int(self.eq_kind), int(self.flags), 0)


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_ptr(t: torch.Tensor, numel: int | None = None, name: str = "tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float64 and t.dtype != torch.uint8:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return t.data_ptr()


class Lattice:
    """One periodic lattice of n nodes.  State tensors are float64 (6, n)."""

    def __init__(self, n: int, params: Params | None = None, stream=None):
        self.n = int(n)
        self.params = params or Params()
        self._h = _vp()
        cp = self.params.c()
        check(lib().lbm_init(ctypes.byref(self._h), self.n, ctypes.byref(cp),
                             _vp(_stream_ptr(stream))))
        self.ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lbm_destroy(h)
            self._h = None

    def set_stream(self, stream=None):
        check(lib().lbm_set_stream(self._h, _vp(_stream_ptr(stream))))

    def set_params(self, params: Params):
        cp = params.c()
        check(lib().lbm_set_params(self._h, ctypes.byref(cp)))
        self.params = params

    def workspace_bytes(self, kind: int = WS_STEP) -> int:
        return int(lib().lbm_workspace_bytes(self._h, kind))

    def workspace(self, device="cuda") -> torch.Tensor:
        nb = self.workspace_bytes(WS_STEP)
        if self.ws is None or self.ws.numel() * 8 < nb:
            self.ws = torch.empty((nb + 7) // 8, dtype=torch.float64,
                                  device=device)
        return self.ws

    def set_tuning(self, kernel=KERNEL_BLOCKED, nodes_per_lane=8,
                   steps_per_launch=40, waves_per_group=4):
        t = CTuning(kernel, nodes_per_lane, steps_per_launch, waves_per_group)
        check(lib().lbm_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = CTuning()
        check(lib().lbm_get_tuning(self._h, ctypes.byref(t)))
        return dict(kernel=t.kernel, nodes_per_lane=t.nodes_per_lane,
                    steps_per_launch=t.steps_per_launch,
                    waves_per_group=t.waves_per_group)

    def equilibrium(self, rho, J, zeta, out: torch.Tensor | None = None):
        n = self.n
        f = out if out is not None else torch.empty(
            (6, n), dtype=torch.float64, device=rho.device)
        check(lib().lbm_set_equilibrium(
            self._h, _dev_ptr(rho, n, "rho"), _dev_ptr(J, n, "J"),
            _dev_ptr(zeta, n, "zeta"), _dev_ptr(f, 6 * n, "f")))
        return f

    def step(self, f: torch.Tensor, nsteps: int, ws: torch.Tensor | None = None):
        """Advances f in place by nsteps time steps."""
        ws = ws if ws is not None else self.workspace(f.device)
        check(lib().lbm_step(self._h, _dev_ptr(f, 6 * self.n, "f"),
                             _dev_ptr(ws, None, "ws"), ws.numel() * 8,
                             int(nsteps)))
        return f

    def step_noalloc(self, f: torch.Tensor, nsteps: int):
        """Advances f in place by nsteps time steps without a workspace
        (lbm_step_noalloc: the library's fixed scratch, n <= NOALLOC_MAX_NODES)."""
        check(lib().lbm_step_noalloc(self._h, _dev_ptr(f, 6 * self.n, "f"),
                                     int(nsteps)))
        return f

    def moments(self, f: torch.Tensor) -> torch.Tensor:
        m = torch.empty_like(f)
        check(lib().lbm_moments(self._h, _dev_ptr(f, 6 * self.n, "f"),
                                _dev_ptr(m, 6 * self.n, "m")))
        return m

    def autotune(self, f: torch.Tensor, probe_steps: int = 64,
                 cache_path: str | None = None) -> dict:
        """Times the candidate tile shapes on f (restored afterwards) and
        keeps the fastest; see lbm_autotune."""
        nb = self.workspace_bytes(WS_TUNE)
        ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=f.device)
        t = CTuning()
        check(lib().lbm_autotune(self._h, _dev_ptr(f, 6 * self.n, "f"),
                                 _dev_ptr(ws), nb, int(probe_steps),
                                 cache_path.encode() if cache_path else None,
                                 ctypes.byref(t)))
        return self.get_tuning()

    # ------------------------------------------------------ gradients --
    def set_adjoint_kernel(self, kernel: int = KERNEL_AUTO):
        check(lib().lbm_set_adjoint_kernel(self._h, int(kernel)))

    def set_recompute_stride(self, stride: int = 0):
        """Stride of the recomputed states the reverse sweep stores (0 auto,
        1 every state, 2 the even ones; lbm_set_recompute_stride)."""
        check(lib().lbm_set_recompute_stride(self._h, int(stride)))

    def adjoint_workspace(self, nsteps: int, ckpt_every: int, device="cuda"):
        nb = int(lib().lbm_adjoint_workspace_bytes(self._h, int(nsteps),
                                                   int(ckpt_every)))
        if nb == 0:
            check(LBM_EINVAL)
        return torch.empty((nb + 7) // 8, dtype=torch.float64, device=device)

    def forward_ckpt(self, f, nsteps: int, ckpt_every: int, aws):
        """Advances f by nsteps steps, keeping checkpoints in aws."""
        check(lib().lbm_forward_ckpt(self._h, _dev_ptr(f, 6 * self.n, "f"),
                                     _dev_ptr(aws), aws.numel() * 8,
                                     int(nsteps), int(ckpt_every)))
        return f

    def adjoint(self, aws, nsteps: int, ckpt_every: int, fbar,
                use_graph: bool = True):
        """fbar: dL/df(T) in, dL/df(0) out.  Returns dL/d(s_e, s_psi, s_eps)."""
        r = (ctypes.c_double * 3)()
        check(lib().lbm_adjoint(self._h, _dev_ptr(aws), aws.numel() * 8,
                                int(nsteps), int(ckpt_every),
                                _dev_ptr(fbar, 6 * self.n, "fbar"), r,
                                1 if use_graph else 0))
        return list(r)

    def loss(self, f, target, aws):
        """L = 1/2 sum (rho - target)^2 (target None: rho0) and dL/df."""
        fbar = torch.empty_like(f)
        L = ctypes.c_double()
        check(lib().lbm_loss(self._h, _dev_ptr(f, 6 * self.n, "f"),
                             None if target is None else _dev_ptr(target, self.n, "target"),
                             _dev_ptr(aws), aws.numel() * 8, ctypes.byref(L),
                             _dev_ptr(fbar)))
        return L.value, fbar

    def equilibrium_adjoint(self, rho, J, zeta, fbar, aws):
        out = [torch.empty_like(rho) for _ in range(3)]
        check(lib().lbm_equilibrium_adjoint(
            self._h, _dev_ptr(rho, self.n), _dev_ptr(J, self.n),
            _dev_ptr(zeta, self.n), _dev_ptr(fbar, 6 * self.n),
            *[_dev_ptr(x) for x in out], _dev_ptr(aws), aws.numel() * 8))
        return tuple(out)

    def moments_adjoint(self, mbar, aws):
        fbar = torch.empty_like(mbar)
        check(lib().lbm_moments_adjoint(self._h, _dev_ptr(mbar, 6 * self.n),
                                        _dev_ptr(fbar), _dev_ptr(aws),
                                        aws.numel() * 8))
        return fbar

    def diagnostics(self, f: torch.Tensor, ws: torch.Tensor | None = None,
                    raise_nonfinite: bool = False):
        ws = ws if ws is not None else self.workspace(f.device)
        out = (ctypes.c_double * 8)()
        rc = lib().lbm_diagnostics(self._h, _dev_ptr(f, 6 * self.n, "f"),
                                   _dev_ptr(ws, None, "ws"), ws.numel() * 8,
                                   out)
        if rc != LBM_OK and (rc != LBM_ENONFINITE or raise_nonfinite):
            check(rc)
        return list(out)


class Batch:
    """Independent periodic lattices of ragged lengths advanced together.

    offsets: int64 sequence of n_inst + 1 boundaries (host); params: one
    Params per lattice.  States are float64 tensors (6, n_total)."""

    def __init__(self, offsets, params, stream=None):
        import numpy as np
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.n_inst = len(self.offsets) - 1
        self.params = list(params)
        if len(self.params) != self.n_inst:
            raise ValueError("need one Params per lattice")
        arr = (CParams * self.n_inst)(*[p.c() for p in self.params])
        self._h = _vp()
        check(lib().lbm_batch_init(
            ctypes.byref(self._h), self.n_inst,
            self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), arr,
            _vp(_stream_ptr(stream))))
        self.n_total = int(lib().lbm_batch_total_nodes(self._h))
        self.ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lbm_batch_destroy(h)
            self._h = None

    def set_stream(self, stream=None):
        check(lib().lbm_batch_set_stream(self._h, _vp(_stream_ptr(stream))))

    def workspace_bytes(self, kind: int = WS_STEP) -> int:
        return int(lib().lbm_batch_workspace_bytes(self._h, kind))

    def _ensure_ws(self, device, kind=WS_STEP):
        nb = self.workspace_bytes(kind)
        if self.ws is None or self.ws.numel() * 8 < nb:
            self.ws = torch.empty((nb + 7) // 8, dtype=torch.float64,
                                  device=device)
        return self.ws

    def set_tuning(self, nodes_per_lane=4, steps_per_launch=16,
                   waves_per_group=4, device="cuda"):
        t = CTuning(KERNEL_BLOCKED, nodes_per_lane, steps_per_launch,
                    waves_per_group)
        check(lib().lbm_batch_set_tuning(self._h, ctypes.byref(t)))
        self.prepare(device)

    def get_tuning(self) -> dict:
        t = CTuning()
        check(lib().lbm_batch_get_tuning(self._h, ctypes.byref(t)))
        return dict(kernel=t.kernel, nodes_per_lane=t.nodes_per_lane,
                    steps_per_launch=t.steps_per_launch,
                    waves_per_group=t.waves_per_group)

    def prepare(self, device="cuda"):
        ws = self._ensure_ws(device)
        check(lib().lbm_batch_prepare(self._h, _dev_ptr(ws), ws.numel() * 8))
        return ws

    def equilibrium(self, rho, J, zeta, out=None):
        n = self.n_total
        ws = self.prepare(rho.device)
        f = out if out is not None else torch.empty(
            (6, n), dtype=torch.float64, device=rho.device)
        check(lib().lbm_batch_set_equilibrium(
            self._h, _dev_ptr(rho, n, "rho"), _dev_ptr(J, n, "J"),
            _dev_ptr(zeta, n, "zeta"), _dev_ptr(f, 6 * n, "f"),
            _dev_ptr(ws), ws.numel() * 8))
        return f

    def run(self, f: torch.Tensor, nsteps: int, use_graph: bool = True):
        ws = self.ws
        if ws is None:
            ws = self.prepare(f.device)
        check(lib().lbm_batch_run(self._h, _dev_ptr(f, 6 * self.n_total, "f"),
                                  _dev_ptr(ws), ws.numel() * 8, int(nsteps),
                                  1 if use_graph else 0))
        return f

    def moments(self, f: torch.Tensor) -> torch.Tensor:
        ws = self.ws if self.ws is not None else self.prepare(f.device)
        m = torch.empty_like(f)
        check(lib().lbm_batch_moments(self._h, _dev_ptr(f, 6 * self.n_total, "f"),
                                      _dev_ptr(m), _dev_ptr(ws), ws.numel() * 8))
        return m

    def diagnostics(self, f: torch.Tensor, raise_nonfinite: bool = False):
        import numpy as np
        ws = self.ws if self.ws is not None else self.prepare(f.device)
        out = np.zeros(8 * self.n_inst)
        rc = lib().lbm_batch_diagnostics(
            self._h, _dev_ptr(f, 6 * self.n_total, "f"), _dev_ptr(ws),
            ws.numel() * 8, out.ctypes.data_as(_dp))
        if rc != LBM_OK and (rc != LBM_ENONFINITE or raise_nonfinite):
            check(rc)
        return out.reshape(self.n_inst, 8)

    def set_groups(self, shapes, group_of=None, device="cuda"):
        """Shape groups of run(): lattice i with shapes[group_of[i]], each
        shape a (P, K, W) triple; no shapes returns to the single tuning."""
        import numpy as np
        n = len(shapes)
        if n == 0:
            check(lib().lbm_batch_set_groups(self._h, 0, None, None))
        else:
            arr = (CTuning * n)(*[CTuning(KERNEL_BLOCKED, int(p), int(k), int(w))
                                  for p, k, w in shapes])
            go = np.ascontiguousarray(np.asarray(group_of, dtype=np.int32))
            if go.shape != (self.n_inst,):
                raise ValueError("group_of needs one entry per lattice")
            check(lib().lbm_batch_set_groups(
                self._h, n, arr, go.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        self.prepare(device)

    def set_resident(self, mode: int = 1, device="cuda"):
        """1: lattices of RESIDENT_MIN..RESIDENT_MAX nodes run all the steps
        of run() in one launch; 0: every lattice in tiles (same results)."""
        check(lib().lbm_batch_set_resident(self._h, int(mode)))
        self.prepare(device)

    def resident_lattices(self) -> int:
        return int(lib().lbm_batch_resident_lattices(self._h))

    def get_groups(self):
        """([(P, K, W), ...], group_of array), or ([], None) without groups."""
        import numpy as np
        n = ctypes.c_int32()
        arr = (CTuning * MAX_GROUPS)()
        go = np.zeros(self.n_inst, dtype=np.int32)
        check(lib().lbm_batch_get_groups(
            self._h, ctypes.byref(n), arr,
            go.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        shapes = [(arr[g].nodes_per_lane, arr[g].steps_per_launch,
                   arr[g].waves_per_group) for g in range(n.value)]
        return shapes, (go if n.value else None)

    def autotune(self, f: torch.Tensor, probe_steps: int = 32,
                 cache_path: str | None = None) -> dict:
        ws = self._ensure_ws(f.device, WS_TUNE)
        t = CTuning()
        check(lib().lbm_batch_autotune(
            self._h, _dev_ptr(f, 6 * self.n_total, "f"), _dev_ptr(ws),
            ws.numel() * 8, int(probe_steps),
            cache_path.encode() if cache_path else None, ctypes.byref(t)))
        return self.get_tuning()

    # ------------------------------------------------------ gradients --
    def set_adjoint_kernel(self, kernel: int = KERNEL_AUTO):
        check(lib().lbm_batch_set_adjoint_kernel(self._h, int(kernel)))

    def set_recompute_stride(self, stride: int = 0):
        check(lib().lbm_batch_set_recompute_stride(self._h, int(stride)))

    def adjoint_workspace(self, nsteps: int, ckpt_every: int, device="cuda"):
        nb = int(lib().lbm_batch_adjoint_workspace_bytes(
            self._h, int(nsteps), int(ckpt_every)))
        if nb == 0:
            check(LBM_EINVAL)
        return torch.empty((nb + 7) // 8, dtype=torch.float64, device=device)

    def forward_ckpt(self, f, nsteps: int, ckpt_every: int, aws):
        check(lib().lbm_batch_forward_ckpt(
            self._h, _dev_ptr(f, 6 * self.n_total, "f"), _dev_ptr(aws),
            aws.numel() * 8, int(nsteps), int(ckpt_every)))
        return f

    def adjoint(self, aws, nsteps: int, ckpt_every: int, fbar,
                use_graph: bool = True):
        """fbar: dL/df(T) in, dL/df(0) out.  Returns (n_inst, 3) rate
        gradients dL_i/d(s_e, s_psi, s_eps) on the device."""
        rbar = torch.empty((self.n_inst, 3), dtype=torch.float64,
                           device=fbar.device)
        check(lib().lbm_batch_adjoint(
            self._h, _dev_ptr(aws), aws.numel() * 8, int(nsteps),
            int(ckpt_every), _dev_ptr(fbar, 6 * self.n_total, "fbar"),
            _dev_ptr(rbar), 1 if use_graph else 0))
        return rbar

    def loss(self, f, target, aws):
        """Per-lattice L_i = 1/2 sum (rho - target)^2 (target None: rho0) on
        the device, and dL/df."""
        fbar = torch.empty_like(f)
        loss = torch.empty(self.n_inst, dtype=torch.float64, device=f.device)
        check(lib().lbm_batch_loss(
            self._h, _dev_ptr(f, 6 * self.n_total, "f"),
            None if target is None else _dev_ptr(target, self.n_total, "target"),
            _dev_ptr(aws), aws.numel() * 8, _dev_ptr(loss), _dev_ptr(fbar)))
        return loss, fbar

    def equilibrium_adjoint(self, rho, J, zeta, fbar, aws):
        out = [torch.empty_like(rho) for _ in range(3)]
        n = self.n_total
        check(lib().lbm_batch_equilibrium_adjoint(
            self._h, _dev_ptr(rho, n), _dev_ptr(J, n), _dev_ptr(zeta, n),
            _dev_ptr(fbar, 6 * n), *[_dev_ptr(x) for x in out], _dev_ptr(aws),
            aws.numel() * 8))
        return tuple(out)

    def moments_adjoint(self, mbar, aws):
        fbar = torch.empty_like(mbar)
        check(lib().lbm_batch_moments_adjoint(
            self._h, _dev_ptr(mbar, 6 * self.n_total), _dev_ptr(fbar),
            _dev_ptr(aws), aws.numel() * 8))
        return fbar
