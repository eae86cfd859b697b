"""Eigenvalues of the Maxwell GEP as a differentiable function of the permittivity.

For a simple eigenvalue lambda of C*C x = lambda B x with B = diag(eps), first-order
perturbation theory gives d lambda / d B_pp = -lambda |x_p|^2 / (x* B x).  The solver returns
x = B^{-1} Q_r Sigma_r y with ||y|| = 1, for which x* B x = lambda, so the derivative is
-|x_p|^2 (per Yee point; per voxel the three Yee points of a grid point are summed).  The
backward pass therefore needs only the eigenvectors of the forward solve and one device
kernel (pcx_grad_eps), whatever the objective: dJ/d eps = sum_t (dJ/d lambda_t) d lambda_t/d eps.

The derivative of an individual eigenvalue inside a degenerate cluster is not defined (only
symmetric functions of the cluster are); objectives should use bands that are simple at the
evaluation point.
"""
from __future__ import annotations

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


class _Eigenvalues:
    """Holder for the torch.autograd.Function (created lazily so that importing this module does
    not import torch)."""
    fn = None


def _function():
    if _Eigenvalues.fn is not None:
        return _Eigenvalues.fn
    torch = _torch()

    class Eigenvalues(torch.autograd.Function):
        @staticmethod
        def forward(ctx, eps, plan, kappa, nev, layout, solve_kwargs):
            host = eps.detach().to(device="cpu", dtype=torch.float64).contiguous().numpy()
            plan.pcx_plan_set_eps(host, layout)
            kw = dict(solve_kwargs or {})
            kw.setdefault("mode", L.PCX_MODE_FP64)
            lam, _, x, _ = plan.pcx_solve(kappa, nev, want_x=True, want_y=True, **kw)
            ctx.plan, ctx.layout = plan, layout
            ctx.eps_shape, ctx.eps_device, ctx.eps_dtype = eps.shape, eps.device, eps.dtype
            ctx.save_for_backward(x)
            return torch.as_tensor(lam, dtype=torch.float64).to(eps.device)

        @staticmethod
        def backward(ctx, g):
            (x,) = ctx.saved_tensors
            w = g.detach().to(device="cpu", dtype=torch.float64).numpy()
            if not np.any(w):
                grad = torch.zeros(ctx.eps_shape, dtype=ctx.eps_dtype, device=ctx.eps_device)
            else:
                grad = ctx.plan.pcx_grad_eps(x, w, ctx.layout)
                grad = grad.reshape(ctx.eps_shape).to(device=ctx.eps_device, dtype=ctx.eps_dtype)
            return grad, None, None, None, None, None

    _Eigenvalues.fn = Eigenvalues
    return Eigenvalues


def eigenvalues(eps, plan, kappa, nev: int, layout: int = L.PCX_EPS_YEE3, **solve_kwargs):
    """The nev smallest positive eigenvalues at wave vector kappa as a torch tensor (float64) that
    carries d lambda / d eps.  eps: torch tensor with 3n values (PCX_EPS_YEE3) or n voxel values
    (PCX_EPS_VOXEL); the plan's permittivity is set from it.  solve_kwargs go to Plan.pcx_solve
    (default mode: FP64)."""
    return _function().apply(eps, plan, kappa, int(nev), int(layout), solve_kwargs)


def band_gap_objective(eps, plan, kappas, lower: int, upper: int, layout: int = L.PCX_EPS_YEE3,
                       **solve_kwargs):
    """J = min_k lambda_upper(k) - max_k lambda_lower(k) (1-based band indices) over the wave
    vectors kappas: the complete gap between two bands, differentiable in eps where the arg-min
    and arg-max are unique."""
    torch = _torch()
    lams = [eigenvalues(eps, plan, k, upper, layout, **solve_kwargs) for k in kappas]
    lam = torch.stack(lams)                          # (nk, upper)
    return lam[:, upper - 1].min() - lam[:, lower - 1].max(), lam
