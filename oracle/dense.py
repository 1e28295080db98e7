"""Dense tier of the oracle: H and S formed explicitly on small grids.

Test infrastructure only (see the package docstring).

Conventions (the paper is silent on the FFT sign and normalisation, Sec. 2.1):
  psi(r_j)      = sum_i c_i exp(+2 pi i g_i . j / n)
  (V_loc psi)_i = n^-3 sum_j exp(-2 pi i g_i . j / n) V_j psi(r_j)
so H_loc[i, k] = Vhat((g_i - g_k) mod n) with Vhat(q) = n^-3 sum_j V_j exp(-2 pi i q . j / n).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def dft_matrix_1d(n: int, sign: int) -> np.ndarray:
    """W[q, j] = exp(sign * 2 pi i q j / n): the textbook DFT matrix, no FFT library involved."""
    q = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(q, q) / n)


def naive_dft3(a: np.ndarray, sign: int) -> np.ndarray:
    """Unnormalised separable 3D DFT by three matrix products (sum_j a_j exp(sign 2 pi i q.j/n))."""
    n = a.shape[0]
    W = dft_matrix_1d(n, sign)
    out = np.einsum("qj,jkl->qkl", W, a)
    out = np.einsum("qk,jkl->jql", W, out)
    return np.einsum("ql,jkl->jkq", W, out)


def vhat(V: np.ndarray) -> np.ndarray:
    """Fourier coefficients of the local potential, Vhat(q) = n^-3 sum_j V_j exp(-2 pi i q.j/n)."""
    n = V.shape[0]
    return naive_dft3(V.astype(np.complex128), -1) / n**3


def h_local(gidx: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Dense V_loc on the sphere: multiplication by V(r) in real space (Sec. 2.1, Alg. 1)."""
    n = V.shape[0]
    vh = vhat(V)
    d = (gidx[:, None, :] - gidx[None, :, :]) % n
    return vh[d[..., 0], d[..., 1], d[..., 2]]


def block_diag(D: list) -> np.ndarray:
    """Block-diagonal D over atoms (Eq. 3: D does not couple different atoms)."""
    if len(D) == 0 or sum(d.shape[0] for d in D) == 0:
        return np.zeros((0, 0))
    return scipy.linalg.block_diag(*D)


def hamiltonian(gidx, kin, V, P, D) -> np.ndarray:
    """H = K + V_loc + P D P^H (Eq. 2 and Eq. 3), complex Hermitian reading of the paper's real form."""
    H = h_local(gidx, V) + np.diag(kin).astype(np.complex128)
    if P.shape[1]:
        H = H + P @ block_diag(D) @ P.conj().T
    return H


def overlap(npw: int, P, Q) -> np.ndarray:
    """S = I + P Q P^H (Eq. 4); S = I for norm-conserving pseudopotentials."""
    S = np.eye(npw, dtype=np.complex128)
    if Q is not None and P.shape[1]:
        S = S + (P * Q[None, :]) @ P.conj().T
    return S


def eig_pencil(H, S):
    """All eigenpairs of H v = lambda S v, ascending, with V^H S V = I (Eq. 1)."""
    return scipy.linalg.eigh(H, S)


def chebyshev_T(m: int, x):
    """Closed form of the degree-m Chebyshev polynomial (Sec. 4.2, c = 0, r = 1):
    cos(m arccos x) on [-1, 1], sign(x)^m cosh(m arccosh |x|) outside."""
    x = np.asarray(x, dtype=np.float64)
    inside = np.abs(x) <= 1.0
    out = np.empty_like(x)
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out


def filter_spectral(H, S, X, m, c, r):
    """T_m((S^-1 H - c)/r) X written through the eigendecomposition of the pencil (Sec. 4.2):
    S^-1 H = V Lambda V^-1 with V^-1 = V^H S, hence T_m(S^-1 H) X = V T_m(Lambda) V^H S X."""
    lam, Vec = eig_pencil(H, S)
    t = chebyshev_T(m, (lam - c) / r)
    return Vec @ (t[:, None] * (Vec.conj().T @ (S @ X)))


def filter_recurrence(H, S, X, m, c, r):
    """Alg. 2 inner loop with the dense operator A = S^-1 H."""
    A = np.linalg.solve(S, H)
    prev = X
    cur = (A @ X - c * X) / r
    for _ in range(2, m + 1):
        prev, cur = cur, (2.0 / r) * (A @ cur - c * cur) - prev
    return cur if m >= 1 else X
