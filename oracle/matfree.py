"""Matrix-free tier of the oracle: Alg. 1 with FFTs, the Woodbury inverse of S, Alg. 2, Rayleigh-Ritz,
the Lanczos upper bound and the outer loop. FP64 throughout; usable at any size (it is also the CPU
baseline of the benchmark).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft
import scipy.linalg

from . import dense


def _workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


class Operators:
    """H, S and S^-1 of the generalized problem H x = lambda S x (Eq. 1-4), never formed.

    gidx (npw, 3) Miller indices; kin (npw,) kinetic diagonal; V (n, n, n) real potential on the grid in
    [x][y][z] order; P (npw, nproj) projectors; D list of per-atom real symmetric blocks (Eq. 3);
    Q (nproj,) overlap coefficients, or None for S = I (Eq. 4).
    """

    def __init__(self, gidx, kin, V, P, D, Q, band_chunk: int = 64, workers: int | None = None):
        self.gidx = np.asarray(gidx)
        self.kin = np.asarray(kin, dtype=np.float64)
        self.V = np.asarray(V, dtype=np.float64)
        self.n = self.V.shape[0]
        self.P = np.asarray(P)
        self.Dfull = dense.block_diag(D).astype(np.complex128)
        self.Q = None if Q is None else np.asarray(Q, dtype=np.float64)
        self.band_chunk = band_chunk
        self.workers = workers or _workers()
        self.idx = tuple((self.gidx % self.n).T)
        if self.Q is not None and self.P.shape[1]:
            # Woodbury (Sec. 5.1): S^-1 = I - P (Q^-1 + P^H P)^-1 P^H; the reduced matrix is factored once
            C = np.diag(1.0 / self.Q).astype(np.complex128) + self.P.conj().T @ self.P
            self.C_chol = scipy.linalg.cho_factor(C)
        else:
            self.C_chol = None

    @classmethod
    def from_problem(cls, pb, **kw):
        return cls(pb.gidx, pb.kin, pb.V, pb.P, pb.D, pb.Q, **kw)

    @property
    def npw(self) -> int:
        return self.gidx.shape[0]

    # --- Alg. 1 pieces -------------------------------------------------------------------------------------
    def vloc(self, psi: np.ndarray) -> np.ndarray:
        """V_loc psi: inverse FFT to real space, multiply by V(r), FFT back (Sec. 2.1, Alg. 1)."""
        psi = np.asarray(psi).reshape(self.npw, -1)
        n = self.n
        out = np.empty_like(psi, dtype=np.complex128)
        for b0 in range(0, psi.shape[1], self.band_chunk):
            b1 = min(psi.shape[1], b0 + self.band_chunk)
            box = np.zeros((b1 - b0, n, n, n), dtype=np.complex128)
            box[(slice(None),) + self.idx] = psi[:, b0:b1].T
            real = scipy.fft.ifftn(box, axes=(1, 2, 3), workers=self.workers) * n**3
            real *= self.V[None]
            back = scipy.fft.fftn(real, axes=(1, 2, 3), workers=self.workers) / n**3
            out[:, b0:b1] = back[(slice(None),) + self.idx].T
        return out

    def project(self, psi):
        """p_psi = P^H psi (Alg. 1)."""
        return self.P.conj().T @ psi

    def apply_H(self, psi):
        """H psi = K psi + V_loc psi + P D_V P^H psi (Alg. 1, Eq. 2-3)."""
        psi = np.asarray(psi, dtype=np.complex128).reshape(self.npw, -1)
        out = self.kin[:, None] * psi + self.vloc(psi)
        if self.P.shape[1]:
            out += self.P @ (self.Dfull @ self.project(psi))
        return out

    def apply_S(self, psi):
        """S psi = psi + P D_S P^H psi (Alg. 1, Eq. 4)."""
        psi = np.asarray(psi, dtype=np.complex128).reshape(self.npw, -1)
        if self.Q is None or not self.P.shape[1]:
            return psi.copy()
        return psi + self.P @ (self.Q[:, None] * self.project(psi))

    def apply_Sinv(self, psi):
        """S^-1 psi by the Woodbury formula (Sec. 5.1), capacitance matrix solved directly in FP64."""
        psi = np.asarray(psi, dtype=np.complex128).reshape(self.npw, -1)
        if self.C_chol is None:
            return psi.copy()
        return psi - self.P @ scipy.linalg.cho_solve(self.C_chol, self.project(psi))

    def apply_A(self, psi):
        """A = S^-1 H, the non-Hermitian operator the filter is a polynomial in (Sec. 4.2)."""
        return self.apply_Sinv(self.apply_H(psi))


# --- Alg. 2 ----------------------------------------------------------------------------------------------
def rayleigh_quotients(ops: Operators, X):
    """Per-band Rayleigh quotients x^H H x / x^H S x (first step of Alg. 2)."""
    HX = ops.apply_H(X)
    SX = ops.apply_S(X)
    return np.real(np.sum(X.conj() * HX, axis=0)) / np.real(np.sum(X.conj() * SX, axis=0))


def chebyshev_filter(ops: Operators, X, m: int, c: float, r: float):
    """psi^0 = X, psi^1 = (A psi^0 - c psi^0)/r, psi^i = 2/r (A psi^(i-1) - c psi^(i-1)) - psi^(i-2),
    returning psi^m unscaled (Alg. 2, recurrence of Sec. 4.2). P^H is recomputed at every step."""
    X = np.asarray(X, dtype=np.complex128)
    if m == 0:
        return X.copy()
    prev = X
    cur = (ops.apply_A(X) - c * X) / r
    for _ in range(2, m + 1):
        prev, cur = cur, (2.0 / r) * (ops.apply_A(cur) - c * cur) - prev
    return cur


def rayleigh_ritz(ops: Operators, Y, with_residuals: bool = True):
    """Subspace matrices H_Y = Y^H H Y, S_Y = Y^H S Y, dense generalized eigenproblem H_Y Z = S_Y Z Lambda
    with Z S_Y-orthonormal, rotation Y <- Y Z (Alg. 2). Returns (ritz ascending, YZ, residual norms)."""
    HY = ops.apply_H(Y)
    SY = ops.apply_S(Y)
    Hs = Y.conj().T @ HY
    Ss = Y.conj().T @ SY
    Hs = 0.5 * (Hs + Hs.conj().T)
    Ss = 0.5 * (Ss + Ss.conj().T)
    lam, Z = scipy.linalg.eigh(Hs, Ss)
    U = Y @ Z
    res = None
    if with_residuals:
        res = np.linalg.norm(HY @ Z - (SY @ Z) * lam[None, :], axis=0)
    return lam, U, res


def residual_norms(ops: Operators, U, lam):
    """||H u_i - lambda_i S u_i||_2 per band (the convergence monitor of Sec. 6.1)."""
    return np.linalg.norm(ops.apply_H(U) - ops.apply_S(U) * lam[None, :], axis=0)


def lanczos_upper_bound(ops: Operators, v0, k: int = 10):
    """k steps of Lanczos on A = S^-1 H in the S inner product (self-adjoint there), from v0.
    Returns (max eigenvalue of the k x k tridiagonal T + the last beta, alphas, betas).

    The paper takes E_cut as the upper edge and notes a few Lanczos steps as the alternative of the
    sequential Chebyshev filtering work it builds on (Sec. 5.3); the Lanczos rule is used here."""
    v = np.asarray(v0, dtype=np.complex128).reshape(-1, 1)
    v = v / np.sqrt(np.real(np.vdot(v, ops.apply_S(v))))
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for _ in range(k):
        Hv = ops.apply_H(v)
        f = ops.apply_Sinv(Hv)
        alpha = float(np.real(np.vdot(v, Hv)))
        f = f - alpha * v - beta * v_prev
        beta = float(np.sqrt(np.real(np.vdot(f, ops.apply_S(f)))))
        alphas.append(alpha)
        betas.append(beta)
        v_prev, v = v, f / beta
    T = np.diag(alphas) + np.diag(betas[:-1], 1) + np.diag(betas[:-1], -1)
    theta = np.linalg.eigvalsh(T)
    return float(theta[-1] + betas[-1]), np.array(alphas), np.array(betas)


def chebfsi(ops: Operators, X0, m: int, iters: int, lam_plus: float, callback=None, lock_tol=None):
    """Outer loop: Rayleigh quotients -> lambda_-, filter centre and radius, filter, Rayleigh-Ritz
    (Alg. 2 repeated; lambda_- is the largest Rayleigh quotient, Sec. 5.3). After a Rayleigh-Ritz step the
    Rayleigh quotients of the rotated block are its Ritz values, so lambda_- is then their maximum.
    With lock_tol, from the second iteration on each band is filtered with the degree the residual estimate
    of Sec. 5.4 (Eq. 5) asks for, at most m (0 = locked); every band stays in the Rayleigh-Ritz step."""
    X = np.asarray(X0, dtype=np.complex128)
    lam_minus = float(np.max(rayleigh_quotients(ops, X)))
    hist = []
    lam = res = None
    for it in range(iters):
        c = 0.5 * (lam_plus + lam_minus)
        r = 0.5 * (lam_plus - lam_minus)
        if lock_tol is not None and hist:
            deg = locking_degrees(res, lam, c, r, m, lock_tol)
            Y = chebyshev_filter_degrees(ops, X, deg, c, r)
        else:
            deg = np.full(X.shape[1], m, dtype=np.int64)
            Y = chebyshev_filter(ops, X, m, c, r)
        lam, X, res = rayleigh_ritz(ops, Y)
        hist.append(dict(it=it, c=c, r=r, lam_minus=lam_minus, ritz=lam.copy(), resid=res.copy(), degrees=deg))
        if callback is not None:
            callback(hist[-1])
        lam_minus = float(np.max(lam))
    return lam, X, res, hist


def stability_factor(m: int, lam1: float, c: float, r: float) -> float:
    """T_m((lambda_1 - c)/r), which must stay far below 1/eps for a well-conditioned S_Y (Sec. 5.3)."""
    return float(dense.chebyshev_T(m, np.array([(lam1 - c) / r]))[0])


# --- locking (Sec. 5.4) ------------------------------------------------------------------------------------
def chebyshev_filter_degrees(ops: Operators, X, degrees, c: float, r: float):
    """Band-wise filter with its own degree per band: column b becomes T_{m_b}((A - c)/r) x_b (Sec. 5.4,
    adaptive degree per band); bands with degree 0 are left unchanged (locked)."""
    X = np.asarray(X, dtype=np.complex128)
    degrees = np.asarray(degrees, dtype=np.int64)
    out = X.copy()
    for m in np.unique(degrees):
        if m == 0:
            continue
        cols = np.nonzero(degrees == m)[0]
        out[:, cols] = chebyshev_filter(ops, X[:, cols], int(m), c, r)
    return out


def locking_degrees(resid, ritz, c: float, r: float, m_max: int, tol: float):
    """Degree per band from the residual estimate of Sec. 5.4 (Eq. 5): after a degree-n filter and
    Rayleigh-Ritz, the residual of band i is about ||r_i|| / |T_n((lambda_i - c)/r)|. The degree is the
    smallest n <= m_max bringing it to tol; a band already at tol is locked (degree 0). The paper's formula
    shows lambda_1 where the text speaks of each band's own lambda_i; the band's own Ritz value is used."""
    resid = np.asarray(resid, dtype=np.float64)
    ritz = np.asarray(ritz, dtype=np.float64)
    deg = np.full(resid.shape, m_max, dtype=np.int64)
    for i in range(resid.shape[0]):
        if resid[i] <= tol:
            deg[i] = 0
            continue
        x = (ritz[i] - c) / r
        for n in range(1, m_max + 1):
            if resid[i] / abs(float(dense.chebyshev_T(n, np.array([x]))[0])) <= tol:
                deg[i] = n
                break
    return deg


# --- capacitance solve by preconditioned iterative refinement (Sec. 5.1) -------------------------------------
def atom_blocks(proj_off):
    """(start, size) of each atom's projector block, from the offsets proj_off[0..natom]."""
    off = np.asarray(proj_off, dtype=np.int64)
    return [(int(off[a]), int(off[a + 1] - off[a])) for a in range(off.shape[0] - 1) if off[a + 1] > off[a]]


def block_preconditioner(C, blocks):
    """M^-1 for M = the atom-block diagonal of C (the preconditioner of Sec. 5.1), as a dense matrix."""
    Minv = np.zeros_like(C)
    for s, n in blocks:
        Minv[s:s + n, s:s + n] = np.linalg.inv(C[s:s + n, s:s + n])
    return Minv


def capacitance_refine(C, blocks, b, iters=None, tol=1e-15, maxit=200):
    """Solve C q = b by iterative refinement preconditioned by the atom-block diagonal M of C (Sec. 5.1):
    q_0 = M^-1 b; r_k = b - C q_k; q_(k+1) = q_k + M^-1 r_k. With iters given, exactly that many corrections;
    otherwise corrections until every column has ||r_k|| <= tol ||b||. Returns (q, corrections, residual
    history: max over columns of ||r_k|| / ||b||)."""
    b = np.asarray(b, dtype=np.complex128)
    b2 = b.reshape(b.shape[0], -1)
    Minv = block_preconditioner(C, blocks)
    q = Minv @ b2
    bn = np.maximum(np.linalg.norm(b2, axis=0), 1e-300)
    hist = []
    k = 0
    while True:
        r = b2 - C @ q
        rel = float(np.max(np.linalg.norm(r, axis=0) / bn))
        hist.append(rel)
        if (iters is not None and k >= iters) or (iters is None and (rel <= tol or k >= maxit)):
            break
        q = q + Minv @ r
        k += 1
    return q.reshape(b.shape), k, np.array(hist)
