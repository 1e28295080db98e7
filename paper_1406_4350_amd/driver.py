"""Outer loop of Chebyshev-filtered subspace iteration on the GPU (Alg. 2, Sec. 5.3).

Host work is limited to scalars: the filter interval [lambda_-, lambda_+] -> centre c and radius r.
Every vector and matrix operation is a call into libchebfd.
"""
from __future__ import annotations

import time

import torch

from .chebfd import Plan


def chebfsi(plan: Plan, X: torch.Tensor, m: int, iters: int, lam_plus: float, callback=None,
            with_residuals: bool = True):
    """Run `iters` outer iterations in place on X (nb, npw). lambda_- is the largest Rayleigh quotient of the
    block: explicitly for the start block, the largest Ritz value afterwards (the Rayleigh quotients of a
    Rayleigh-Ritz-rotated block are its Ritz values). Returns (ritz, residuals, history)."""
    lam_minus = float(plan.rayleigh_quotients(X).max().item())
    hist = []
    ritz = res = None
    for it in range(iters):
        if not lam_plus > lam_minus:
            raise ValueError(f"upper bound {lam_plus} not above lambda_- {lam_minus}")
        c = 0.5 * (lam_plus + lam_minus)
        r = 0.5 * (lam_plus - lam_minus)
        t0 = time.perf_counter()
        plan.filter(X, m, c, r)
        ritz, res = plan.rayleigh_ritz(X, with_residuals=with_residuals)
        torch.cuda.synchronize()
        rec = dict(it=it, c=c, r=r, lam_minus=lam_minus, seconds=time.perf_counter() - t0,
                   ritz=ritz.cpu().numpy(), resid=None if res is None else res.cpu().numpy())
        hist.append(rec)
        if callback is not None:
            callback(rec)
        lam_minus = float(rec["ritz"].max())
    return ritz, res, hist
