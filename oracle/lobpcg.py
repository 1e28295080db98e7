"""LOBPCG oracle: the block method the paper compares the Chebyshev filter with (Sec. 2.3, "Block algorithms:
LOBPCG"), for the same generalized problem H x = lambda S x, in FP64 with the matrix-free operators.

One iteration is a Rayleigh-Ritz step in the space spanned by the current Ritz vectors X, the preconditioned
residuals W and the previous search directions P (3 nb columns; 2 nb on the first iteration). The lowest nb
Ritz pairs become the new X, and the part of the update outside X becomes the new P. Products with H and S of
the new vectors are carried by the same linear combinations, so every iteration applies H and S to W only.

The preconditioner damps high kinetic energies (Sec. 2.2 describes it as a smooth rational function of the
kinetic energy, thresholded at the kinetic energy of the band); the rational function used is the one of the
conjugate-gradient method the paper cites (Payne et al., 1992):
    K(x) = (27 + 18 x + 12 x^2 + 8 x^3) / (27 + 18 x + 12 x^2 + 8 x^3 + 16 x^4),  x = t_G / E_kin(band).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .matfree import Operators


def tpa(x):
    """The rational preconditioner function K(x) above; K(0) = 1 and K(x) ~ 1 / (2x) for large x."""
    x = np.asarray(x, dtype=np.float64)
    num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x))
    return num / (num + 16.0 * x**4)


def precondition(kin, X, R):
    """W = K(t / E_kin) R column by column, with E_kin = x^H K x / x^H x of the band's current vector."""
    ekin = np.real(np.sum(kin[:, None] * np.abs(X) ** 2, axis=0)) / np.real(np.sum(np.abs(X) ** 2, axis=0))
    return tpa(kin[:, None] / ekin[None, :]) * R


TRUNC = 1e-14  # relative eigenvalue cut of the scaled Gram matrix


def _rr(V, HV, SV, nb):
    """Lowest nb Ritz pairs of the pencil (V^H H V, V^H S V) in an S-orthonormal basis of span(V): near
    convergence W and P become almost dependent on X and V^H S V singular to working precision, so the basis is
    taken from the eigendecomposition of the diagonally scaled Gram matrix, dropping directions whose
    eigenvalue is below TRUNC times the largest (SVQB basis of Stathopoulos and Wu). Returns (lam, C) with
    V C the Ritz vectors."""
    A = V.conj().T @ HV
    B = V.conj().T @ SV
    A = 0.5 * (A + A.conj().T)
    B = 0.5 * (B + B.conj().T)
    d = 1.0 / np.sqrt(np.real(np.diag(B)))
    sig, U = np.linalg.eigh(d[:, None] * B * d[None, :])
    keep = sig > TRUNC * sig[-1]
    Q = d[:, None] * U[:, keep] / np.sqrt(sig[keep])[None, :]
    As = Q.conj().T @ A @ Q
    lam, Y = np.linalg.eigh(0.5 * (As + As.conj().T))
    return lam[:nb], Q @ Y[:, :nb]


def lobpcg(ops: Operators, X0, iters: int, precond: bool = True, active_tol: float = 1e-8, restart: int = 10,
           callback=None):
    """Full-block LOBPCG from the start block X0 (npw x nb). Returns (ritz, X, residual norms, history).
    history[k] holds the Ritz values after iteration k, the residual norms ||H x - lambda S x|| of the vectors
    that entered iteration k (iteration 0 = the Rayleigh-Ritz of X0) and the number of active bands.

    Bands whose residual is <= active_tol contribute no W or P columns (soft locking at the target
    tolerance): the corrections of converged bands are nearly dependent on X, and keeping them makes the Gram
    matrix singular and the carried products H V, S V drift until the iteration diverges (observed below
    residuals of about 1e-9 with this basis). The band itself stays in X and in every Rayleigh-Ritz.

    Every `restart` iterations H X and S X are recomputed from X and the directions dropped for that iteration
    (a restart of the recurrence), which bounds the drift of the carried products."""
    X = np.asarray(X0, dtype=np.complex128)
    nb = X.shape[1]
    # start: Rayleigh-Ritz of X0
    HX, SX = ops.apply_H(X), ops.apply_S(X)
    lam, C = _rr(X, HX, SX, nb)
    X, HX, SX = X @ C, HX @ C, SX @ C
    hist = [dict(it=0, ritz=lam.copy(), resid=None, active=nb)]
    P = HP = SP = None
    for it in range(1, iters + 1):
        if restart and it > 1 and (it - 1) % restart == 0:
            HX, SX = ops.apply_H(X), ops.apply_S(X)
            P = HP = SP = None
        R = HX - SX * lam[None, :]
        res = np.linalg.norm(R, axis=0)
        act = np.nonzero(res > active_tol)[0]
        W = precondition(ops.kin, X[:, act], R[:, act]) if precond else R[:, act]
        HW, SW = ops.apply_H(W), ops.apply_S(W)
        blocks = [(X, HX, SX), (W, HW, SW)]
        if P is not None:
            blocks.append((P[:, act], HP[:, act], SP[:, act]))
        V, HV, SV = (np.hstack([b[j] for b in blocks]) for j in range(3))
        lam, C = _rr(V, HV, SV, nb)
        Cx, Cr = C[:nb], C[nb:]
        P, HP, SP = V[:, nb:] @ Cr, HV[:, nb:] @ Cr, SV[:, nb:] @ Cr
        X, HX, SX = X @ Cx + P, HX @ Cx + HP, SX @ Cx + SP
        hist.append(dict(it=it, ritz=lam.copy(), resid=res, active=int(act.size)))
        if callback is not None:
            callback(hist[-1])
    res = np.linalg.norm(HX - SX * lam[None, :], axis=0)
    return lam, X, res, hist
