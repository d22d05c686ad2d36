"""torch.autograd.Function wrappers of the forward run and its hand-written
adjoint (library calls lbm_forward_ckpt / lbm_adjoint and their batch forms).

LBMFunction.apply(rho0, J0, zeta0, s_e, s_eps, nsteps, ckpt_every, consts)
returns the density field after nsteps time steps from the equilibrium
initial state (rho0, J0, zeta0).  s_psi is coupled to s_e as in section 7 of
the paper (sigma_psi = (3/2)(gamma/Pr) sigma_e); the library returns the
partial derivatives with respect to the three rates and the chain rule
through s_psi(s_e) is applied here on the host (a scalar product), so the
gradient of s_e is the total one.
"""
from __future__ import annotations

import torch

from . import lbm


def _consts(consts: dict | None) -> dict:
    c = dict(lam=1.0, rho0=1.0, cp=1.0, gamma=1.4, prandtl=1.0, c0=0.5, s0=0.0,
             source_on=1)
    c.update(consts or {})
    return c


def _rate_like(value, like):
    """A rate gradient as a tensor on the device and of the shape of the rate
    it belongs to."""
    return torch.as_tensor(value, dtype=torch.float64).to(like.device).reshape(like.shape)


class LBMFunction(torch.autograd.Function):
    """s_e and s_eps may be Python numbers (no gradient) or 0-d tensors on
    any device (gradients on the same device)."""

    @staticmethod
    def forward(ctx, rho0, J0, zeta0, s_e, s_eps, nsteps: int, ckpt_every: int,
                consts: dict | None = None):
        c = _consts(consts)
        for name, r in (("s_e", s_e), ("s_eps", s_eps)):
            if torch.is_tensor(r) and r.numel() != 1:
                raise ValueError(f"LBMFunction: {name} must be a number or a "
                                 f"one-element tensor, got shape {tuple(r.shape)}")
        ctx.rate_like = tuple(r.detach() if torch.is_tensor(r) else None
                              for r in (s_e, s_eps))
        se = float(s_e)
        s_psi, _, dpsi = lbm.coupled_rates(se, c["gamma"], c["prandtl"])
        p = lbm.Params(s_e=se, s_psi=s_psi, s_eps=float(s_eps), **c)
        n = rho0.numel()
        lat = lbm.Lattice(n, p)
        rho0, J0, zeta0 = (x.detach().contiguous() for x in (rho0, J0, zeta0))
        f = lat.equilibrium(rho0, J0, zeta0)
        aws = lat.adjoint_workspace(nsteps, ckpt_every, rho0.device)
        lat.forward_ckpt(f, nsteps, ckpt_every, aws)
        rho_T = lat.moments(f)[0].clone()
        ctx.lat, ctx.aws, ctx.dpsi = lat, aws, dpsi
        ctx.nsteps, ctx.ckpt = int(nsteps), int(ckpt_every)
        ctx.save_for_backward(rho0, J0, zeta0)
        return rho_T

    @staticmethod
    def backward(ctx, grad_rho):
        rho0, J0, zeta0 = ctx.saved_tensors
        lat, aws = ctx.lat, ctx.aws
        mbar = torch.zeros((6, lat.n), dtype=torch.float64, device=rho0.device)
        mbar[0] = grad_rho
        fbar = lat.moments_adjoint(mbar, aws)
        r = lat.adjoint(aws, ctx.nsteps, ctx.ckpt, fbar)
        g_rho, g_J, g_zeta = lat.equilibrium_adjoint(rho0, J0, zeta0, fbar, aws)
        like_se, like_seps = ctx.rate_like
        g_se = (_rate_like(r[0] + r[1] * ctx.dpsi, like_se)
                if ctx.needs_input_grad[3] else None)
        g_seps = (_rate_like(r[2], like_seps)
                  if ctx.needs_input_grad[4] else None)
        return g_rho, g_J, g_zeta, g_se, g_seps, None, None, None


class BatchLBMFunction(torch.autograd.Function):
    """Batch form: rho0, J0, zeta0 are (n_total,) fields in the batch layout
    of `offsets`; s_e and s_eps are (n_inst,) tensors on any device (their
    gradients come back on the same device).  Returns the (n_total,) density
    after nsteps."""

    @staticmethod
    def forward(ctx, rho0, J0, zeta0, s_e, s_eps, offsets, nsteps: int,
                ckpt_every: int, consts: dict | None = None):
        c = _consts(consts)
        n_inst = len(offsets) - 1
        for name, r in (("s_e", s_e), ("s_eps", s_eps)):
            if not torch.is_tensor(r) or r.shape != (n_inst,):
                raise ValueError(f"BatchLBMFunction: {name} must be a tensor of "
                                 f"shape ({n_inst},), one rate per lattice")
        ctx.rate_like = (s_e.detach(), s_eps.detach())
        se = s_e.detach().cpu().tolist()
        seps = s_eps.detach().cpu().tolist()
        params, dpsi = [], []
        for a, b in zip(se, seps):
            s_psi, _, d = lbm.coupled_rates(a, c["gamma"], c["prandtl"])
            params.append(lbm.Params(s_e=a, s_psi=s_psi, s_eps=b, **c))
            dpsi.append(d)
        bt = lbm.Batch(offsets, params)
        rho0, J0, zeta0 = (x.detach().contiguous() for x in (rho0, J0, zeta0))
        f = bt.equilibrium(rho0, J0, zeta0)
        aws = bt.adjoint_workspace(nsteps, ckpt_every, rho0.device)
        bt.forward_ckpt(f, nsteps, ckpt_every, aws)
        rho_T = bt.moments(f)[0].clone()
        ctx.bt, ctx.aws = bt, aws
        ctx.dpsi = torch.tensor(dpsi, dtype=torch.float64, device=rho0.device)
        ctx.nsteps, ctx.ckpt = int(nsteps), int(ckpt_every)
        ctx.save_for_backward(rho0, J0, zeta0)
        return rho_T

    @staticmethod
    def backward(ctx, grad_rho):
        rho0, J0, zeta0 = ctx.saved_tensors
        bt, aws = ctx.bt, ctx.aws
        mbar = torch.zeros((6, bt.n_total), dtype=torch.float64,
                           device=rho0.device)
        mbar[0] = grad_rho
        fbar = bt.moments_adjoint(mbar, aws)
        r = bt.adjoint(aws, ctx.nsteps, ctx.ckpt, fbar)
        g_rho, g_J, g_zeta = bt.equilibrium_adjoint(rho0, J0, zeta0, fbar, aws)
        like_se, like_seps = ctx.rate_like
        g_se = (_rate_like(r[:, 0] + r[:, 1] * ctx.dpsi, like_se)
                if ctx.needs_input_grad[3] else None)
        g_seps = (_rate_like(r[:, 2], like_seps)
                  if ctx.needs_input_grad[4] else None)
        return g_rho, g_J, g_zeta, g_se, g_seps, None, None, None, None
