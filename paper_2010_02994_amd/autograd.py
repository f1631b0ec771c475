"""Hand-written adjoint of the Hawkes log-likelihood behind torch.autograd.

The forward pass calls the C ABI once (hawkes_grad), which returns the
log-likelihood together with its exact gradient with respect to the N x D
locations (App. A of arXiv 2010.02994) and the six parameters; both are saved,
and backward scales them by the incoming gradient.  This is what an HMC
leapfrog step needs (Sec. 3.3): one call yields ell and grad ell.

Double backward is not supported (the Hessian is not implemented).
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import api


class HawkesLoglik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, params: torch.Tensor, t: torch.Tensor, prec: str = "mixed"):
        """x: (N, D) device tensor (float64 or float32); params: (6,) tensor in the
        order (mu, h, tau, theta, omega, xi); t: (N,) float64 device tensor, sorted.
        Returns the log-likelihood as a 0-d float64 tensor on x's device."""
        if params.numel() != 6:
            raise ValueError("params must have 6 entries (mu, h, tau, theta, omega, xi)")
        x64 = x.detach().to(torch.float64).contiguous()
        t64 = t.detach().to(torch.float64).contiguous()
        p = params.detach().to("cpu", torch.float64).reshape(6)
        ll, gx, gp = api.grad(x64, t64, p.tolist(), prec=prec)
        ctx.x_dtype = x.dtype
        ctx.p_meta = (params.dtype, params.device, params.shape)
        ctx.save_for_backward(gx, torch.as_tensor(gp, dtype=torch.float64))
        return torch.tensor(ll, dtype=torch.float64, device=x.device)

    @staticmethod
    @once_differentiable
    def backward(ctx, g: torch.Tensor):
        gx, gp = ctx.saved_tensors
        dtype, device, shape = ctx.p_meta
        gxo = (gx * g.to(gx.device)).to(ctx.x_dtype) if ctx.needs_input_grad[0] else None
        gpo = (gp.to(device) * g.to(device)).to(dtype).reshape(shape) if ctx.needs_input_grad[1] else None
        return gxo, gpo, None, None


def hawkes_loglik(x: torch.Tensor, params: torch.Tensor, t: torch.Tensor, prec: str = "mixed") -> torch.Tensor:
    """Differentiable log-likelihood ell(x, params; t)."""
    return HawkesLoglik.apply(x, params, t, prec)


class BmdsLoglik(torch.autograd.Function):
    """Bayesian MDS log-likelihood of the latent locations (Sec. 2.2.3) with its
    hand-written adjoint: one library call returns ell, d ell/d sigma and
    d ell/d x.  With `hawkes_loglik` on the same x this gives the influenza
    model's log density over the locations and its gradient (Sec. 3)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, sigma: torch.Tensor, delta: torch.Tensor, prec: str = "fp64"):
        """x: (N, D) device tensor; sigma: scalar tensor (> 0); delta: (N, N)
        float64 device tensor (strict lower triangle read, NaN = unobserved).
        Returns ell as a 0-d float64 tensor on x's device (no host sync)."""
        x64 = x.detach().to(torch.float64).contiguous()
        s = float(sigma.detach().reshape(()).item())
        out4, gx = api.bmds(x64, delta.detach().to(torch.float64).contiguous(), s, prec=prec)
        ctx.x_dtype = x.dtype
        ctx.s_meta = (sigma.dtype, sigma.device, sigma.shape)
        ctx.save_for_backward(gx, out4)
        return out4[0].clone()

    @staticmethod
    @once_differentiable
    def backward(ctx, g: torch.Tensor):
        gx, out4 = ctx.saved_tensors
        dtype, device, shape = ctx.s_meta
        gxo = (gx * g.to(gx.device)).to(ctx.x_dtype) if ctx.needs_input_grad[0] else None
        gso = (out4[1].to(device) * g.to(device)).to(dtype).reshape(shape) if ctx.needs_input_grad[1] else None
        return gxo, gso, None, None


def bmds_loglik(x: torch.Tensor, sigma: torch.Tensor, delta: torch.Tensor, prec: str = "fp64") -> torch.Tensor:
    """Differentiable MDS log-likelihood ell(x, sigma; delta)."""
    return BmdsLoglik.apply(x, sigma, delta, prec)
