"""Gamma-point oracle: real wavefunctions (Sec. 2.1 takes the wavefunctions real) stored on the half sphere.

A real function has c_-G = conj c_G, so it is fixed by the coefficients on the half sphere H+. The stored
vector holds sqrt(2) c_G for G != 0 and the real c_0 at G = 0: then the Euclidean inner product of two stored
vectors, real part, equals the inner product of the functions on the whole sphere. Every operator here is the
full-sphere operator of `matfree` between an expansion and a contraction, so it is exact whenever the
full-sphere operators map real functions to real functions (projectors real in real space).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from . import matfree


class GammaMap:
    """Expansion of half-sphere vectors to the whole sphere and back."""

    def __init__(self, gidx_full, half):
        gidx_full = np.asarray(gidx_full)
        self.half = np.asarray(half)
        self.npw_full = gidx_full.shape[0]
        pos = {tuple(g): i for i, g in enumerate(gidx_full)}
        self.mirror = np.array([pos[tuple(-g)] for g in gidx_full[self.half]])
        self.zero = np.all(gidx_full[self.half] == 0, axis=1)
        self.scale = np.where(self.zero, 1.0, np.sqrt(2.0))

    def expand(self, Y):
        """c_G = y_G / sqrt(2) (G != 0), c_0 = y_0, c_-G = conj c_G."""
        Y = np.asarray(Y, dtype=np.complex128).reshape(self.half.shape[0], -1)
        c = Y / self.scale[:, None]
        out = np.zeros((self.npw_full, Y.shape[1]), dtype=np.complex128)
        out[self.mirror] = np.conj(c)
        out[self.half] = c
        return out

    def contract(self, C):
        """Half-sphere coefficients of a full-sphere vector (its real-function part)."""
        C = np.asarray(C, dtype=np.complex128).reshape(self.npw_full, -1)
        c = 0.5 * (C[self.half] + np.conj(C[self.mirror]))
        return c * self.scale[:, None]


class GammaOperators:
    """H, S, S^-1 on half-sphere vectors through the full-sphere matrix-free operators."""

    def __init__(self, full_ops: matfree.Operators, gmap: GammaMap):
        self.full = full_ops
        self.map = gmap
        self.kin = full_ops.kin[gmap.half]

    @classmethod
    def from_problem(cls, gp):
        return cls(matfree.Operators.from_problem(gp.full), GammaMap(gp.full.gidx, gp.half))

    def apply_H(self, Y):
        return self.map.contract(self.full.apply_H(self.map.expand(Y)))

    def apply_S(self, Y):
        return self.map.contract(self.full.apply_S(self.map.expand(Y)))

    def apply_Sinv(self, Y):
        return self.map.contract(self.full.apply_Sinv(self.map.expand(Y)))

    def apply_A(self, Y):
        return self.apply_Sinv(self.apply_H(Y))


def dense_real(ops: GammaOperators, which: str = "H"):
    """The operator as a real symmetric matrix in the real basis [Re y; Im y] of the half-sphere vectors
    (the imaginary part at G = 0 dropped): size = number of plane waves of the whole sphere."""
    nh = ops.map.half.shape[0]
    keep_im = ~ops.map.zero
    cols = []
    f = {"H": ops.apply_H, "S": ops.apply_S}[which]
    for k in range(nh):
        e = np.zeros(nh, dtype=np.complex128)
        e[k] = 1.0
        cols.append(f(e)[:, 0])
    for k in np.nonzero(keep_im)[0]:
        e = np.zeros(nh, dtype=np.complex128)
        e[k] = 1j
        cols.append(f(e)[:, 0])
    Y = np.array(cols).T
    return np.vstack([Y.real, Y.imag[keep_im]])


def chebyshev_filter(ops: GammaOperators, Y, m, c, r):
    """The recurrence of Alg. 2 on half-sphere vectors."""
    Y = np.asarray(Y, dtype=np.complex128)
    if m == 0:
        return Y.copy()
    prev, cur = Y, (ops.apply_A(Y) - c * Y) / r
    for _ in range(2, m + 1):
        prev, cur = cur, (2.0 / r) * (ops.apply_A(cur) - c * cur) - prev
    return cur


def rayleigh_ritz(ops: GammaOperators, Y):
    """Rayleigh-Ritz with the real parts of the subspace matrices (the inner products of real functions);
    real eigenvectors, so the rotated vectors stay real functions. Returns (ritz, YZ, residual norms)."""
    HY, SY = ops.apply_H(Y), ops.apply_S(Y)
    Hs = np.real(Y.conj().T @ HY)
    Ss = np.real(Y.conj().T @ SY)
    Hs, Ss = 0.5 * (Hs + Hs.T), 0.5 * (Ss + Ss.T)
    import scipy.linalg

    lam, Z = scipy.linalg.eigh(Hs, Ss)
    res = np.linalg.norm(HY @ Z - (SY @ Z) * lam[None, :], axis=0)
    return lam, Y @ Z, res


def rayleigh_quotients(ops: GammaOperators, Y):
    return np.real(np.sum(Y.conj() * ops.apply_H(Y), axis=0)) / np.real(np.sum(Y.conj() * ops.apply_S(Y), axis=0))


def chebfsi(ops: GammaOperators, X0, m, iters, lam_plus):
    """The outer loop of matfree.chebfsi on half-sphere vectors."""
    X = np.asarray(X0, dtype=np.complex128)
    lam_minus = float(np.max(rayleigh_quotients(ops, X)))
    hist = []
    for it in range(iters):
        c, r = 0.5 * (lam_plus + lam_minus), 0.5 * (lam_plus - lam_minus)
        lam, X, res = rayleigh_ritz(ops, chebyshev_filter(ops, X, m, c, r))
        hist.append(dict(it=it, c=c, r=r, lam_minus=lam_minus, ritz=lam.copy(), resid=res.copy()))
        lam_minus = float(np.max(lam))
    return lam, X, res, hist
