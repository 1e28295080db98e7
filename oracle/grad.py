"""Adjoint of one Chebyshev filter + Rayleigh-Ritz pass (an addition beyond the paper; the forward steps are
Alg. 2 with the recurrence of Sec. 4.2). FP64, matrix-free.

Test infrastructure only (see the package docstring).

Loss: L = sum_{i < nk} w_i lambda_i over the lowest nk Ritz values of Y = T_m((S^-1 H - c)/r) X0, with c and
r held fixed. Differentiated with respect to X0 (complex), V(r) (real, on the grid) and the real symmetric
per-atom blocks D_a. Convention for the complex gradient G of a real loss: dL = 2 Re tr(G^H dX).

  Rayleigh-Ritz: dlambda_i = z_i^H (dH_Y - lambda_i dS_Y) z_i (non-degenerate lambda_i, Z^H S_Y Z = I), so
     through H at fixed Y:   dL/dV_j  += n^-3 sum_i w_i |u_i(r_j)|^2,  dL/dD_kl += sum_i w_i Re(conj(p_ik) p_il)
     through Y:              Ybar = sum_i w_i (H u_i - lambda_i S u_i) z_i^H,  u_i = Y z_i,  p_i = P^H u_i
  Filter (psi^i = s_i (A - c) psi^(i-1) - t_i psi^(i-2), A = S^-1 H, s_1 = 1/r, t_1 = 0, s_i = 2/r, t_i = 1):
     a = S^-1 psibar^i;  psibar^(i-1) += s_i (H a - c psibar^i);  psibar^(i-2) -= t_i psibar^i
     dL/dV_j  += 2 s_i n^-3 Re sum_b conj(a_b(r_j)) psi_b^(i-1)(r_j)
     dL/dD_kl += s_i Re sum_b [conj(Pa)_bk (P psi^(i-1))_bl + conj(Pa)_bl (P psi^(i-1))_bk]
  dL/dX0 = psibar^0.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg

from . import matfree


def real_space(ops: matfree.Operators, psi: np.ndarray) -> np.ndarray:
    """psi(r_j) = sum_i c_i exp(+2 pi i g_i.j/n) for each column, shape (nb, n, n, n)."""
    n = ops.n
    box = np.zeros((psi.shape[1], n, n, n), dtype=np.complex128)
    box[(slice(None),) + ops.idx] = psi.T
    return scipy.fft.ifftn(box, axes=(1, 2, 3), workers=ops.workers) * n**3


def block_entries(D: list):
    """Index pairs (k, l) of the block-diagonal entries, in the packed order of the D blocks."""
    rows, cols = [], []
    off = 0
    for d in D:
        na = d.shape[0]
        for k in range(na):
            for l in range(na):
                rows.append(off + k)
                cols.append(off + l)
        off += na
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)


def loss(ops: matfree.Operators, X0, m, c, r, w):
    """L = sum_i w_i lambda_i of the lowest len(w) Ritz values after one filter + Rayleigh-Ritz pass."""
    Y = matfree.chebyshev_filter(ops, X0, m, c, r)
    lam = matfree.rayleigh_ritz(ops, Y, with_residuals=False)[0]
    return float(np.dot(w, lam[: len(w)]))


def filter_rr_grad(ops: matfree.Operators, X0, m: int, c: float, r: float, w, D: list):
    """Returns (L, ritz, dX0, dV (n, n, n) in [x][y][z] order, dD packed like the D blocks)."""
    X0 = np.asarray(X0, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    nk = w.shape[0]
    n = ops.n
    # forward, keeping every iterate
    psis = [X0]
    if m >= 1:
        psis.append((ops.apply_A(X0) - c * X0) / r)
    for _ in range(2, m + 1):
        psis.append((2.0 / r) * (ops.apply_A(psis[-1]) - c * psis[-1]) - psis[-2])
    Y = psis[m]
    HY, SY = ops.apply_H(Y), ops.apply_S(Y)
    Hs = Y.conj().T @ HY
    Ss = Y.conj().T @ SY
    lam, Z = scipy.linalg.eigh(0.5 * (Hs + Hs.conj().T), 0.5 * (Ss + Ss.conj().T))
    L = float(np.dot(w, lam[:nk]))
    ZK = Z[:, :nk]
    U = Y @ ZK
    R = HY @ ZK - (SY @ ZK) * lam[None, :nk]
    Ybar = (R * w[None, :]) @ ZK.conj().T

    rows, cols = block_entries(D)
    dV = np.zeros((n, n, n))
    dD = np.zeros(rows.shape[0])
    # Hellmann-Feynman terms of the Rayleigh-Ritz step
    ur = real_space(ops, U)
    dV += np.einsum("b,bxyz->xyz", w, np.abs(ur) ** 2) / n**3
    if ops.P.shape[1]:
        pu = ops.P.conj().T @ U
        dD += np.real(np.einsum("b,kb,lb->kl", w, pu.conj(), pu))[rows, cols]

    # reverse recurrence
    bar = [np.zeros_like(X0) for _ in range(m + 1)]
    bar[m] = Ybar
    for i in range(m, 0, -1):
        s = (1.0 if i == 1 else 2.0) / r
        a = ops.apply_Sinv(bar[i])
        bar[i - 1] = bar[i - 1] + s * (ops.apply_H(a) - c * bar[i])
        if i >= 2:
            bar[i - 2] = bar[i - 2] - bar[i]
        ar = real_space(ops, a)
        pr = real_space(ops, psis[i - 1])
        dV += 2.0 * s * np.real(np.sum(ar.conj() * pr, axis=0)) / n**3
        if ops.P.shape[1]:
            pa = ops.P.conj().T @ a
            pp = ops.P.conj().T @ psis[i - 1]
            G = np.real(pa.conj() @ pp.T)
            dD += s * (G + G.T)[rows, cols]
    return L, lam, bar[0], dV, dD
