"""Differentiable Geodesic Sinkhorn distance (torch.autograd.Function).

Forward runs Algorithm 1 through gs_sinkhorn, recording every iteration's
floored denominators (ckpt_every = GS_RECORD_ALL, 2 * iters * n * B floats)
or checkpointing w every ckpt_every iterations; backward calls the library's
hand-written reverse sweep gs_sinkhorn_backward, which reads the records (or
recomputes each checkpoint segment) and applies the adjoint Chebyshev
recurrence (p_K is symmetric, so the adjoint of an application is another
application, with a second accumulator for the derivative in t).
"""
from __future__ import annotations

import numpy as np
import torch

from .api import GS_RECORD_ALL, Plan, ckpt_floats, gs_sinkhorn, gs_sinkhorn_backward


class GeoSinkhornDistance(torch.autograd.Function):
    """D_b = 4t sum a (mu_b ln v_b + nu_b ln w_b) for the plan's B pairs.

    apply(mu, nu, t, plan, lambda_hat, iters, ckpt_every=GS_RECORD_ALL, phi=1e-30, a=None)
      mu, nu: (n, B) float32 device tensors; t: float or 0-dim tensor.
    Returns a (B,) float64 tensor on mu's device.  Gradients flow to mu, nu
    (on their supports; zero elsewhere) and to t when it is a tensor that
    requires grad.
    """

    @staticmethod
    def forward(ctx, mu, nu, t, plan: Plan, lambda_hat: float, iters: int, ckpt_every: int = GS_RECORD_ALL,
                phi: float = 1e-30, a=None):
        tval = float(t.detach().item()) if isinstance(t, torch.Tensor) else float(t)
        mu_c = mu.detach().contiguous()
        nu_c = nu.detach().contiguous()
        ckpt = torch.empty(ckpt_floats(plan, iters, ckpt_every), device=mu.device, dtype=torch.float32)
        out = gs_sinkhorn(plan, lambda_hat, tval, mu_c, nu_c, iters, phi=phi, a=a, ckpt_every=ckpt_every,
                          ckpt=ckpt)
        ctx.save_for_backward(mu_c, nu_c, ckpt)
        t_meta = (t.shape, t.dtype, t.device) if isinstance(t, torch.Tensor) else None
        ctx.cfg = (plan, lambda_hat, tval, iters, ckpt_every, phi, a, t_meta)
        return torch.as_tensor(out["dist"], device=mu.device)

    @staticmethod
    def backward(ctx, grad_D):
        mu, nu, ckpt = ctx.saved_tensors
        plan, lam, tval, iters, ce, phi, a, t_meta = ctx.cfg
        t_is_tensor = t_meta is not None
        g = np.asarray(grad_D.detach().double().cpu().numpy(), dtype=np.float64).reshape(-1)
        need_mu, need_nu, need_t = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gmu = torch.empty_like(mu) if need_mu else None
        gnu = torch.empty_like(nu) if need_nu else None
        gt = gs_sinkhorn_backward(plan, lam, tval, mu, nu, iters, ce, ckpt, g, phi=phi, a=a, grad_mu=gmu,
                                  grad_nu=gnu, want_grad_t=bool(need_t and t_is_tensor))
        grad_t = None
        if need_t and t_is_tensor:
            # autograd requires t's own device, dtype and shape
            grad_t = torch.full(t_meta[0], float(np.sum(gt)), dtype=t_meta[1], device=t_meta[2])
        return gmu, gnu, grad_t, None, None, None, None, None, None


def geodesic_sinkhorn_distance(mu, nu, t, plan: Plan, lambda_hat: float, iters: int, ckpt_every: int = GS_RECORD_ALL,
                               phi: float = 1e-30, a=None):
    """Functional form of GeoSinkhornDistance.apply."""
    return GeoSinkhornDistance.apply(mu, nu, t, plan, lambda_hat, iters, ckpt_every, phi, a)
