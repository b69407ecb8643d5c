"""torch.autograd.Function over the C ABI: E2(c, E0) with the screening mask
held at the forward point.

forward  -> shci_pt2_det        (E2)
backward -> shci_pt2_grad       (dE2/dc_i = sum_a 2 H_ai A_a / D_a,
                                 dE2/dE0  = -sum_a A_a^2 / D_a^2; the adjoint
                                 regenerates the connections of every i)

The semistochastic form E2 = E2_det(eps2_d) + mean_s [S_s(eps2) - S_s(eps2_d)]
adds shci_pt2_sample / shci_pt2_sample_grad on fixed draws (draws, p_i and
masks held at the forward point).
"""
from __future__ import annotations

import torch

from .binding import Context


class PT2Function(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, e0, pt2: Context, dets, eps2: float, precision: str = "fp64"):
        e0v = float(e0)
        r = pt2.det(dets, c.detach(), e0v, eps2, precision)
        ctx.pt2 = pt2
        ctx.eps2 = eps2
        ctx.precision = precision
        ctx.e0 = e0v
        ctx.save_for_backward(c.detach(), dets)
        return torch.tensor(r.e2, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, gout):
        c, dets = ctx.saved_tensors
        _, g, de0, _ = ctx.pt2.grad(dets, c, ctx.e0, ctx.eps2, ctx.precision)
        gc = g * gout
        ge0 = gout * de0
        return gc, ge0, None, None, None, None


def pt2_energy(pt2: Context, dets, c, e0, eps2, precision="fp64"):
    """Differentiable E2; `c` and `e0` may require grad (e0 a 0-d float64 tensor)."""
    if not torch.is_tensor(e0):
        e0 = torch.tensor(float(e0), dtype=torch.float64, device=c.device)
    return PT2Function.apply(c, e0, pt2, dets, eps2, precision)


class SemistochasticPT2Function(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, e0, pt2: Context, dets, eps2: float, eps2_d: float, draws, precision: str = "fp64"):
        e0v = float(e0)
        rd = pt2.det(dets, c.detach(), e0v, eps2_d, precision)
        _, mean, _, _ = pt2.sample(dets, c.detach(), e0v, eps2, eps2_d, draws, precision)
        ctx.pt2 = pt2
        ctx.eps = (eps2, eps2_d)
        ctx.precision = precision
        ctx.e0 = e0v
        ctx.save_for_backward(c.detach(), dets, draws)
        return torch.tensor(rd.e2 + mean, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, gout):
        c, dets, draws = ctx.saved_tensors
        eps2, eps2_d = ctx.eps
        _, gd, de0d, _ = ctx.pt2.grad(dets, c, ctx.e0, eps2_d, ctx.precision)
        _, _, _, gs, de0s, _ = ctx.pt2.sample_grad(dets, c, ctx.e0, eps2, eps2_d, draws, ctx.precision)
        return (gd + gs) * gout, gout * (de0d + de0s), None, None, None, None, None, None


def pt2_semistochastic_energy(pt2: Context, dets, c, e0, eps2, eps2_d, draws, precision="fp64"):
    """Differentiable semistochastic E2 on fixed draws [n_samples, n_draws]."""
    if not torch.is_tensor(e0):
        e0 = torch.tensor(float(e0), dtype=torch.float64, device=c.device)
    return SemistochasticPT2Function.apply(c, e0, pt2, dets, eps2, eps2_d, draws, precision)
