"""Outer loop of Chebyshev-filtered subspace iteration on the GPU (Alg. 2, Sec. 5.3).

Host work is limited to scalars: the filter interval [lambda_-, lambda_+] -> centre c and radius r.
Every vector and matrix operation is a call into libchebfd.
"""
from __future__ import annotations

import math
import time

import torch

from .chebfd import Plan, locking_degrees


def chebyshev_magnitude(m: int, x: float) -> float:
    """|T_m(x)| from the closed form: cos(m arccos x) inside [-1, 1], cosh(m arccosh |x|) outside (host scalar)."""
    if abs(x) <= 1.0:
        return abs(math.cos(m * math.acos(x)))
    t = m * math.acosh(abs(x))
    return math.inf if t > 709.0 else math.cosh(t)


def chebfsi(plan: Plan, X: torch.Tensor, m: int, iters: int, lam_plus: float, callback=None,
            with_residuals: bool = True, lock_tol: float | None = None, carry: bool = False):
    """Run `iters` outer iterations in place on X (nb, npw). lambda_- is the largest Rayleigh quotient of the
    block: explicitly for the start block, the largest Ritz value afterwards (the Rayleigh quotients of a
    Rayleigh-Ritz-rotated block are its Ritz values). With lock_tol, after each Rayleigh-Ritz step every band
    gets the degree the residual estimate of Eq. 5 asks for to reach lock_tol with the next filter (at most m,
    0 = locked; Sec. 5.4); the first iteration uses m for all bands. With carry, Rayleigh-Ritz returns the
    projections P^H X and (K + V) X of the rotated block and the next filter starts from them instead of
    recomputing them (see cheb_filter_carry). Each history record
    also carries the amplification T_m((lambda_1 - c)/r) of the lowest band (lambda_1: the lowest Ritz value so
    far, the lowest Rayleigh quotient before the first Rayleigh-Ritz step), which must stay far below 1/eps of
    the band precision for the filtered block to stay well conditioned (Sec. 5.3). Returns (ritz, residuals,
    history)."""
    if lock_tol is not None and not with_residuals:
        raise ValueError("locking needs the residuals")
    rq = plan.rayleigh_quotients(X)
    lam_minus = float(rq.max().item())
    lam_low = float(rq.min().item())
    hist = []
    ritz = res = None
    nb = X.shape[0]
    # carry: Rayleigh-Ritz hands the projections and (K + V) X of its rotated block to the next filter
    # (cheb_rayleigh_ritz_carry, cheb_filter_carry), which then does not compute them
    pc = plan.projections(nb) if carry and plan.nproj > 0 else None
    hx = torch.empty((nb, X.shape[1]), dtype=X.dtype, device=X.device) if carry else None
    have = False
    for it in range(iters):
        if not lam_plus > lam_minus:
            raise ValueError(f"upper bound {lam_plus} not above lambda_- {lam_minus}")
        c = 0.5 * (lam_plus + lam_minus)
        r = 0.5 * (lam_plus - lam_minus)
        degrees = nlocked = None
        if lock_tol is not None and hist:
            degrees, nlocked = locking_degrees(hist[-1]["ritz"], hist[-1]["resid"], c, r, m, lock_tol)
        t0 = time.perf_counter()
        if degrees is None:
            plan.filter(X, m, c, r, p_in=pc if have else None, hx_in=hx if have else None)
        else:
            plan.filter_degrees(X, degrees, c, r)
        ritz, res = plan.rayleigh_ritz(X, with_residuals=with_residuals, p_out=pc, hx_out=hx)
        have = carry
        torch.cuda.synchronize()
        rec = dict(it=it, c=c, r=r, lam_minus=lam_minus, seconds=time.perf_counter() - t0,
                   stability=chebyshev_magnitude(m, (lam_low - c) / r),
                   ritz=ritz.cpu().numpy(), resid=None if res is None else res.cpu().numpy(),
                   band_applications=nb * m if degrees is None else int(degrees.sum()),
                   locked=0 if degrees is None else nlocked, degrees=None if degrees is None else degrees.copy())
        hist.append(rec)
        if callback is not None:
            callback(rec)
        lam_minus = float(rec["ritz"].max())
        lam_low = min(lam_low, float(rec["ritz"].min()))
    return ritz, res, hist


def lobpcg(plan: Plan, X: torch.Tensor, iters: int, tol: float = 1e-8, callback=None):
    """Full-block LOBPCG (Sec. 2.3) in place on X (nb, npw): the start Rayleigh-Ritz and `iters` iterations.
    Bands with residual <= tol add no correction (soft locking). Returns (ritz, history); history[k] has the
    Ritz values after iteration k and the residuals of the vectors that entered it (None for k = 0)."""
    nb = X.shape[0]
    state = plan.lobpcg_state(nb)
    ritz = torch.zeros(nb, dtype=torch.float64, device=X.device)
    hist = []
    for it in range(iters + 1):
        t0 = time.perf_counter()
        res, nact = plan.lobpcg_iterate(X, it, tol, state, ritz)
        torch.cuda.synchronize()
        rec = dict(it=it, ritz=ritz.cpu().numpy(), resid=None if it == 0 else res.cpu().numpy(), active=nact,
                   seconds=time.perf_counter() - t0)
        hist.append(rec)
        if callback is not None:
            callback(rec)
        if it > 0 and nact == 0:
            break
    return ritz, hist
