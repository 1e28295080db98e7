"""torch.autograd wrapper of one Chebyshev filter + Rayleigh-Ritz pass (the differentiation form).

ritz = ChebFilterRR.apply(X0, V, D, plan, m, c, r, ckpt_every) returns the nb Ritz values (ascending) of
T_m((S^-1 H - c)/r) X0 for the potential V (n^3, FP64) and the packed D blocks; c and r are constants.
Gradients flow to X0, V and D through the library's hand-written adjoint (cheb_filter_rr_backward). Torch
expects, for a complex leaf, twice the G of dL = 2 Re tr(G^H dX0); the factor is applied here.
"""
from __future__ import annotations

import torch

from .chebfd import Plan


class ChebFilterRR(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X0, V, D, plan: Plan, m: int, c: float, r: float, ckpt_every: int = 3):
        plan.set_potential(V.detach())
        plan.set_D(D.detach())
        Y = X0.detach().clone()
        plan.filter(Y, m, c, r)
        ritz, _ = plan.rayleigh_ritz(Y, with_residuals=False)
        ctx.save_for_backward(X0.detach(), V.detach(), D.detach())
        ctx.plan, ctx.args = plan, (m, c, r, ckpt_every)
        return ritz

    @staticmethod
    def backward(ctx, g):
        X0, V, D = ctx.saved_tensors
        plan = ctx.plan
        m, c, r, k = ctx.args
        g = g.detach().to(torch.float64)
        nz = torch.nonzero(g).flatten()
        nk = int(nz.max().item()) + 1 if nz.numel() else 1
        plan.set_potential(V)
        plan.set_D(D)
        _, dX, dV, dD = plan.filter_rr_backward(X0, m, c, r, g[:nk], k)
        return 2.0 * dX, dV.to(V.device, V.dtype), dD.to(D.device, D.dtype), None, None, None, None, None
