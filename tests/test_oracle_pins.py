"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics, not by the oracle itself.

Each test names what it pins. The mutation tests at the end plant plausible mistakes in the oracle (on the
CPU) and check that some pin catches each one.
"""
import numpy as np
import pytest
import scipy.linalg

from conftest import golden
from oracle import dense, matfree
from paper_1406_4350_amd import workload as wl


@pytest.fixture(scope="module")
def tiny():
    pb = wl.make_problem("tiny_paw")
    H = dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D)
    S = dense.overlap(pb.npw, pb.P, pb.Q)
    return pb, H, S, matfree.Operators.from_problem(pb)


@pytest.fixture(scope="module")
def nc16():
    pb = wl.make_problem("nc16")
    H = dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D)
    S = dense.overlap(pb.npw, pb.P, pb.Q)
    return pb, H, S, matfree.Operators.from_problem(pb)


# ---- basis -------------------------------------------------------------------------------------------------
def test_sphere_sizes():
    """|g| <= R inclusive: 257 / 7153 / 57777 / 17077 / 137065 plane waves for R = 4, 12, 24, 16, 32."""
    for R, npw in [(4, 257), (12, 7153), (24, 57777), (16, 17077), (32, 137065)]:
        g = wl.sphere(R)
        assert g.shape == (npw, 3)
        assert np.all((g.astype(np.int64) ** 2).sum(1) <= R * R)
        key = (g[:, 0] * 1000 + g[:, 1]) * 1000 + g[:, 2]
        assert np.all(np.diff(key) > 0)  # column-sorted, then gz ascending


def test_free_electron_spectrum():
    """V = 0, no projectors: eigenvalues are the kinetic shells 1/2 |2 pi g/L|^2 (Sec. 2.1), golden table."""
    fe = wl.free_electron("nc16")
    H = dense.hamiltonian(fe.gidx, fe.kin, fe.V, fe.P, fe.D)
    lam = np.linalg.eigvalsh(H)
    rows = golden("free_electron_L10_R4.txt")
    start = 0
    for s, mult, val in rows[:5]:
        blk = lam[start:start + int(mult)]
        assert np.allclose(blk, val, atol=1e-14, rtol=0)
        start += int(mult)
    assert abs(lam[-1] - rows[-1][2]) < 1e-14
    assert lam.size == 257


# ---- FFT convention ------------------------------------------------------------------------------------------
def test_naive_dft_matches_library_fft():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(12, 12, 12)) + 1j * rng.normal(size=(12, 12, 12))
    assert np.allclose(dense.naive_dft3(a, -1), np.fft.fftn(a), atol=1e-11)
    assert np.allclose(dense.naive_dft3(a, +1), np.fft.ifftn(a) * 12**3, atol=1e-11)


def test_parseval_and_single_plane_wave():
    n = 16
    g = wl.sphere(4)
    rng = np.random.default_rng(1)
    c = rng.normal(size=g.shape[0]) + 1j * rng.normal(size=g.shape[0])
    box = np.zeros((n, n, n), complex)
    box[tuple((g % n).T)] = c
    real = dense.naive_dft3(box, +1)
    assert abs(np.sum(np.abs(real) ** 2) - n**3 * np.sum(np.abs(c) ** 2)) < 1e-9 * n**3 * np.sum(np.abs(c) ** 2)
    # a single plane wave is a pure phase in real space and a delta after the forward transform
    box = np.zeros((n, n, n), complex)
    box[1, 2, n - 3] = 1.0
    real = dense.naive_dft3(box, +1)
    assert np.allclose(np.abs(real), 1.0, atol=1e-13)
    back = dense.naive_dft3(real, -1) / n**3
    assert np.allclose(back, box, atol=1e-13)


def test_constant_potential_shifts_spectrum(nc16):
    """V = V0: V_loc = V0 I, so every eigenvalue of H moves by V0."""
    pb, H, S, _ = nc16
    V0 = -0.731
    Hl = dense.h_local(pb.gidx, np.full_like(pb.V, V0))
    assert np.allclose(Hl, V0 * np.eye(pb.npw), atol=1e-13)
    ops = matfree.Operators(pb.gidx, pb.kin, np.full_like(pb.V, V0), pb.P, pb.D, pb.Q)
    ops0 = matfree.Operators(pb.gidx, pb.kin, np.zeros_like(pb.V), pb.P, pb.D, pb.Q)
    assert np.allclose(ops.apply_H(pb.X0) - ops0.apply_H(pb.X0), V0 * pb.X0, atol=1e-12)


def test_hloc_structure(nc16):
    """Hermitian, depends only on g_i - g_k, trace = Npw mean(V)."""
    pb = nc16[0]
    Hl = dense.h_local(pb.gidx, pb.V)
    assert np.allclose(Hl, Hl.conj().T, atol=1e-14)
    assert abs(np.trace(Hl) - pb.npw * pb.V.mean()) < 1e-11
    g = pb.gidx
    diff = {}
    for i in range(0, pb.npw, 7):
        for k in range(0, pb.npw, 5):
            key = tuple(g[i] - g[k])
            if key in diff:
                assert abs(Hl[i, k] - diff[key]) < 1e-14
            diff[key] = Hl[i, k]


# ---- operators ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["nc16", "tiny"])
def test_matrix_free_equals_dense(which, request):
    pb, H, S, ops = request.getfixturevalue(which)
    X = pb.X0[:, :5]
    assert np.allclose(ops.apply_H(X), H @ X, atol=1e-12)
    assert np.allclose(ops.apply_S(X), S @ X, atol=1e-13)
    assert np.allclose(ops.apply_Sinv(X), np.linalg.solve(S, X), atol=1e-12)
    assert np.allclose(H, H.conj().T, atol=1e-14)
    assert np.allclose(S, S.conj().T, atol=1e-14)


def test_nonlocal_spectrum(tiny):
    """Nonzero eigenvalues of P D P^H equal the eigenvalues of D (P^H P) (Eq. 3)."""
    pb = tiny[0]
    Dn = dense.block_diag(pb.D)
    big = np.linalg.eigvalsh(pb.P @ Dn @ pb.P.conj().T)
    small = np.sort(np.linalg.eigvals(Dn @ (pb.P.conj().T @ pb.P)).real)
    big_nz = np.sort(big[np.argsort(np.abs(big))[-pb.nproj:]])
    assert np.allclose(big_nz, small, atol=1e-12)
    assert np.sum(np.abs(big) > 1e-10) <= pb.nproj


def test_overlap_spectrum_and_woodbury(tiny):
    """spec(S) = {1 (Npw - Nprojs times)} U 1 + spec(Q^1/2 P^H P Q^1/2) (Eq. 4); S S^-1 = I (Sec. 5.1)."""
    pb, _, S, ops = tiny
    lam = np.linalg.eigvalsh(S)
    q = np.sqrt(pb.Q)
    small = 1.0 + np.linalg.eigvalsh(q[:, None] * (pb.P.conj().T @ pb.P) * q[None, :])
    expect = np.sort(np.concatenate([np.ones(pb.npw - pb.nproj), small]))
    assert np.allclose(lam, expect, atol=1e-13)
    X = pb.X0[:, :4]
    assert np.allclose(S @ ops.apply_Sinv(X), X, atol=1e-12)
    assert np.all(lam > 0)


# ---- Chebyshev filter ---------------------------------------------------------------------------------------
def test_chebyshev_scalars_fig2():
    """Fig. 2 setting: damped [0, 2] -> c = 1, r = 1; the recurrence (Sec. 4.2) run on a diagonal operator
    must give the tabulated values, the closed form too, and T_m(+-1) = (+-1)^m, |T_m| <= 1 inside."""
    rows = np.array(golden("chebyshev_fig2.txt"))
    x, t4 = rows[:, 0], rows[:, 1]
    H = np.diag(x).astype(complex)
    out = dense.filter_recurrence(H, np.eye(len(x)), np.eye(len(x), dtype=complex), 4, 1.0, 1.0)
    assert np.allclose(np.diag(out).real, t4, atol=1e-12)
    assert np.allclose(dense.chebyshev_T(4, x - 1.0), t4, atol=1e-12)
    for m in range(0, 9):
        assert np.allclose(dense.chebyshev_T(m, np.array([1.0, -1.0])), [1.0, (-1.0) ** m])
        assert np.all(np.abs(dense.chebyshev_T(m, np.linspace(-1, 1, 101))) <= 1 + 1e-14)


@pytest.mark.parametrize("m", [1, 2, 5])
def test_filter_matches_spectral_form(tiny, m):
    """T_m(S^-1 H) X = V T_m(Lambda) V^H S X (Sec. 4.2) for the non-Hermitian S^-1 H of a PAW pencil."""
    pb, H, S, ops = tiny
    lam = dense.eig_pencil(H, S)[0]
    c = 0.5 * (lam[-1] + lam[10])
    r = 0.5 * (lam[-1] - lam[10])
    X = pb.X0[:, :6]
    ref = dense.filter_spectral(H, S, X, m, c, r)
    scale = np.linalg.norm(ref)
    assert np.linalg.norm(dense.filter_recurrence(H, S, X, m, c, r) - ref) < 1e-12 * scale
    assert np.linalg.norm(matfree.chebyshev_filter(ops, X, m, c, r) - ref) < 1e-12 * scale


# ---- Rayleigh-Ritz ----------------------------------------------------------------------------------------------
def test_rayleigh_ritz_properties(tiny):
    pb, H, S, ops = tiny
    exact = dense.eig_pencil(H, S)[0]
    Y = pb.X0[:, :10]
    lam, U, res = matfree.rayleigh_ritz(ops, Y)
    assert np.all(lam >= exact[:10] - 1e-12)                       # Courant-Fischer
    assert np.allclose(U.conj().T @ S @ U, np.eye(10), atol=1e-11)  # S-orthonormal rotation
    assert np.allclose(res, np.linalg.norm(H @ U - (S @ U) * lam, axis=0), atol=1e-11)
    M = np.random.default_rng(3).normal(size=(10, 10)) + 1j * np.random.default_rng(4).normal(size=(10, 10))
    lam2 = matfree.rayleigh_ritz(ops, Y @ M)[0]                     # span invariance
    assert np.allclose(lam, lam2, atol=1e-10)
    ev = dense.eig_pencil(H, S)[1][:, :7] @ M[:7, :7]              # exact invariant subspace
    lam3, _, res3 = matfree.rayleigh_ritz(ops, ev)
    assert np.allclose(lam3, exact[:7], atol=1e-12)
    assert np.all(res3 < 1e-10)


def _rq_pin_failures(rq, ops, H, S, X):
    """Failures of a Rayleigh-quotient routine rq(ops, X) against facts of the pencil (first step of Alg. 2):
    the quotient of an exact eigenvector is its eigenvalue; quotients do not change when a column is scaled by
    a complex number; every quotient lies in [lambda_1, lambda_max]."""
    lam, V = dense.eig_pencil(H, S)
    bad = []
    cols = [0, 1, 7, len(lam) // 2, len(lam) - 1]
    q = rq(ops, V[:, cols])
    if not np.allclose(q, lam[cols], rtol=0, atol=1e-12 * max(1.0, np.abs(lam).max())):
        bad.append("eigenvector quotients differ from the eigenvalues")
    s = np.exp(1j * np.arange(X.shape[1])) * np.logspace(-3, 3, X.shape[1])
    q1, q2 = rq(ops, X), rq(ops, X * s[None, :])
    if not np.allclose(q1, q2, rtol=1e-12, atol=1e-12):
        bad.append("not invariant under column scaling")
    if not (np.all(q1 >= lam[0] - 1e-12) and np.all(q1 <= lam[-1] + 1e-12)):
        bad.append("quotient outside [lambda_1, lambda_max]")
    return bad


def test_rayleigh_quotients_pins(tiny, nc16):
    """Pins of matfree.rayleigh_quotients (first step of Alg. 2) on a PAW pencil (S != I) and an S = I one."""
    for pb, H, S, ops in (tiny, nc16):
        assert _rq_pin_failures(matfree.rayleigh_quotients, ops, H, S, pb.X0) == []


def _krylov_ritz(H, S, v0, k):
    """Ritz values of the pencil on span{v0, A v0, ..., A^(k-1) v0}, A = S^-1 H, from an S-orthonormal basis
    built by Arnoldi with two Gram-Schmidt passes (dense matrices; no Lanczos three-term shortcut). Returns
    (Ritz values ascending, coefficient vectors of the basis)."""
    A = np.linalg.solve(S, H)
    V = np.zeros((H.shape[0], k), dtype=np.complex128)
    v = np.asarray(v0, dtype=np.complex128)
    V[:, 0] = v / np.sqrt(np.real(v.conj() @ S @ v))
    for j in range(1, k):
        w = A @ V[:, j - 1]
        for _ in range(2):
            w = w - V[:, :j] @ (V[:, :j].conj().T @ (S @ w))
        V[:, j] = w / np.sqrt(np.real(w.conj() @ S @ w))
    th, Y = scipy.linalg.eigh(V.conj().T @ H @ V, V.conj().T @ S @ V)
    return th, Y, V, A


def _lanczos_pin_failures(lanczos, ops, H, S, v0):
    """Failures of a Lanczos routine lanczos(ops, v0, k) -> (bound, alphas, betas) on A = S^-1 H in the S inner
    product (Sec. 5.3): the eigenvalues of T_k are the Rayleigh-Ritz values of the pencil on the Krylov space
    (computed independently above) and lie in [lambda_1, lambda_max]; the last beta times the last component
    of T_k's top eigenvector is the S-norm of the top Ritz pair's residual A x - theta x; the bound of k = 10
    steps is >= lambda_max; and with k = 80 on a 257-dimensional pencil (top gap 2e-3 .. 2e-2 Ha here) the top
    Ritz value has converged to lambda_max."""
    lam = dense.eig_pencil(H, S)[0]
    bad = []
    for k in range(1, 11):
        bound, al, be = lanczos(ops, v0, k)
        T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
        th, Y = np.linalg.eigh(T)
        thr, Yr, V, A = _krylov_ritz(H, S, v0, k)
        if not np.allclose(th, thr, rtol=0, atol=1e-9 * max(1.0, np.abs(lam).max())):
            bad.append(f"k={k}: T_k eigenvalues differ from the Krylov Ritz values")
        if th.min() < lam[0] - 1e-10 or th.max() > lam[-1] + 1e-10:
            bad.append(f"k={k}: T_k eigenvalue outside the spectrum")
        x = V @ Yr[:, -1]
        rr = A @ x - thr[-1] * x
        rnorm = np.sqrt(np.real(rr.conj() @ S @ rr))
        if abs(be[-1] * abs(Y[-1, -1]) - rnorm) > 1e-8 * max(1.0, rnorm):
            bad.append(f"k={k}: last beta does not give the top Ritz residual")
        if k == 10 and bound < lam[-1]:
            bad.append("k=10: bound below lambda_max")
    _, al, be = lanczos(ops, v0, 80)
    th80 = np.linalg.eigvalsh(np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1))
    if abs(th80.max() - lam[-1]) > 1e-8 * max(1.0, abs(lam[-1])):
        bad.append("k=80: top Ritz value not converged to lambda_max")
    return bad


def test_lanczos_upper_bound(tiny, nc16):
    """Pins of matfree.lanczos_upper_bound (Sec. 5.3) on a PAW pencil and an S = I one."""
    for pb, H, S, ops in (tiny, nc16):
        lmax = dense.eig_pencil(H, S)[0][-1]
        lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
        assert lmax <= lp < lmax + 2.0
        assert _lanczos_pin_failures(matfree.lanczos_upper_bound, ops, H, S, pb.v0) == []


def test_driver_converges_to_pencil(tiny):
    """Bands whose residual has converged carry the exact eigenvalues of the pencil (Sec. 6.1 monitor)."""
    pb, H, S, ops = tiny
    exact = dense.eig_pencil(H, S)[0]
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lam, U, res, hist = matfree.chebfsi(ops, pb.X0, pb.cfg.m, pb.cfg.iters, lp)
    conv = res < 1e-7
    assert conv.sum() >= 8
    assert np.all(np.abs(lam[conv] - exact[:pb.cfg.nb][conv]) < 1e-10)
    # lambda_- of the next iteration is the largest Ritz value, an upper estimate of lambda_nb
    assert hist[-1]["lam_minus"] >= exact[pb.cfg.nb - 1] - 1e-12
    assert matfree.stability_factor(pb.cfg.m, lam[0], hist[-1]["c"], hist[-1]["r"]) < 1e8


# ---- planted mistakes (the pins above must catch them) -------------------------------------------------------
def test_planted_sign_error_in_fft_is_caught(tiny, monkeypatch):
    pb, H, S, ops = tiny
    bad = matfree.Operators.from_problem(pb)
    real_vloc = bad.vloc

    def wrong_vloc(psi):  # conjugated potential phase: equivalent to a wrong FFT sign on one side
        return np.conj(real_vloc(np.conj(psi)))
    monkeypatch.setattr(bad, "vloc", wrong_vloc)
    assert not np.allclose(bad.apply_H(pb.X0[:, :3]), H @ pb.X0[:, :3], atol=1e-12)


def test_planted_transposed_projection_is_caught(tiny):
    pb, H, S, ops = tiny
    bad = matfree.Operators.from_problem(pb)
    bad.Dfull = bad.Dfull.T + 0.1 * np.triu(np.ones_like(bad.Dfull.real), 1)  # non-symmetric D
    assert not np.allclose(bad.apply_H(pb.X0[:, :3]), H @ pb.X0[:, :3], atol=1e-12)


def test_planted_recurrence_error_is_caught(tiny, monkeypatch):
    pb, H, S, ops = tiny
    lam = dense.eig_pencil(H, S)[0]
    c, r = 0.5 * (lam[-1] + lam[10]), 0.5 * (lam[-1] - lam[10])
    X = pb.X0[:, :3]
    ref = dense.filter_spectral(H, S, X, 4, c, r)

    def bad_filter(ops, X, m, c, r):  # psi^1 with 2/r instead of 1/r
        prev, cur = X, (2.0 / r) * (ops.apply_A(X) - c * X)
        for _ in range(2, m + 1):
            prev, cur = cur, (2.0 / r) * (ops.apply_A(cur) - c * cur) - prev
        return cur
    assert np.linalg.norm(bad_filter(ops, X, 4, c, r) - ref) > 1e-6 * np.linalg.norm(ref)


def test_planted_rayleigh_quotient_error_is_caught(tiny):
    """Dividing by x^H x instead of x^H S x (S forgotten in the denominator) fails the quotient pins."""
    pb, H, S, ops = tiny

    def bad_rq(ops, X):
        HX = ops.apply_H(X)
        return np.real(np.sum(X.conj() * HX, axis=0)) / np.real(np.sum(X.conj() * X, axis=0))
    assert _rq_pin_failures(bad_rq, ops, H, S, pb.X0) != []


def test_planted_euclidean_lanczos_is_caught(tiny):
    """Lanczos on S^-1 H with Euclidean inner products (the S inner product forgotten) fails the Lanczos pins."""
    pb, H, S, ops = tiny

    def bad_lanczos(ops, v0, k=10):
        v = np.asarray(v0, dtype=np.complex128).reshape(-1, 1)
        v = v / np.linalg.norm(v)
        v_prev, beta, al, be = np.zeros_like(v), 0.0, [], []
        for _ in range(k):
            f = ops.apply_A(v)
            alpha = float(np.real(np.vdot(v, f)))
            f = f - alpha * v - beta * v_prev
            beta = float(np.linalg.norm(f))
            al.append(alpha)
            be.append(beta)
            v_prev, v = v, f / beta
        T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
        return float(np.linalg.eigvalsh(T)[-1] + be[-1]), np.array(al), np.array(be)
    assert _lanczos_pin_failures(bad_lanczos, ops, H, S, pb.v0) != []


def test_planted_woodbury_error_is_caught(tiny):
    pb, H, S, ops = tiny
    C = np.diag(pb.Q).astype(complex) + pb.P.conj().T @ pb.P  # Q instead of Q^-1
    bad = pb.X0[:, :2] - pb.P @ np.linalg.solve(C, pb.P.conj().T @ pb.X0[:, :2])
    assert not np.allclose(S @ bad, pb.X0[:, :2], atol=1e-8)


# ---- locking (Sec. 5.4) --------------------------------------------------------------------------------------
def test_filter_degrees_reduces_to_filter(tiny):
    pb, H, S, ops = tiny
    lam = dense.eig_pencil(H, S)[0]
    c, r = 0.5 * (lam[-1] + lam[10]), 0.5 * (lam[-1] - lam[10])
    X = pb.X0[:, :6]
    full = matfree.chebyshev_filter(ops, X, 4, c, r)
    assert np.allclose(matfree.chebyshev_filter_degrees(ops, X, [4] * 6, c, r), full, atol=1e-12 * np.abs(full).max())
    deg = [0, 3, 1, 4, 0, 2]
    out = matfree.chebyshev_filter_degrees(ops, X, deg, c, r)
    for b, m in enumerate(deg):  # spectral form T_m(S^-1 H) x_b, band by band
        want = X[:, b] if m == 0 else dense.filter_spectral(H, S, X[:, [b]], m, c, r)[:, 0]
        assert np.allclose(out[:, b], want, atol=1e-11 * max(np.abs(want).max(), 1.0))


def test_locking_degree_rule():
    """Degree = smallest n with ||r|| / |T_n((lambda - c)/r)| <= tol (Eq. 5), 0 when already converged."""
    c, r = 2.0, 1.0
    # x = (lambda - c)/r = -3: |T_n(-3)| = 3, 17, 99, 577, ...
    res = np.array([1e-9, 1e-6 * 3.5, 1e-6 * 16, 1e-6 * 600, 1.0])
    lam = np.full(5, -1.0)
    deg = matfree.locking_degrees(res, lam, c, r, 6, 1e-6)
    assert list(deg) == [0, 2, 2, 5, 6]
    assert abs(dense.chebyshev_T(2, np.array([-3.0]))[0] - 17.0) < 1e-12


@pytest.fixture(scope="module")
def mid_run():
    pb = wl.make_problem("mid_paw")
    ops = matfree.Operators.from_problem(pb)
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    return pb, ops, lp


def test_locking_estimate_becomes_exact(mid_run):
    """Eq. 5 is exact at convergence: once the block has converged for a few iterations, the residual after
    the next degree-m iteration is within a factor 2 of ||r_i|| / |T_m((lambda_i - c)/r)| for the wanted
    bands (residuals far above rounding). Using lambda_1 for every band instead fails this."""
    pb, ops, lp = mid_run
    hist = matfree.chebfsi(ops, pb.X0, pb.cfg.m, 7, lp)[3]
    nw = pb.cfg.nb - 8
    for h0, h1 in zip(hist[4:-1], hist[5:]):
        c, r = h1["c"], h1["r"]
        est = h0["resid"] / np.abs(dense.chebyshev_T(pb.cfg.m, (h0["ritz"] - c) / r))
        keep = h1["resid"][:nw] > 1e-9
        assert keep.sum() > nw // 2
        ratio = h1["resid"][:nw][keep] / est[:nw][keep]
        assert np.all((ratio > 0.5) & (ratio < 2.0)), ratio
        est1 = h0["resid"] / np.abs(dense.chebyshev_T(pb.cfg.m, (h0["ritz"][0] - c) / r))
        assert np.any(h1["resid"][:nw][keep] / est1[:nw][keep] > 2.0)


def test_locking_outer_loop(mid_run):
    """With locking, the wanted eigenpairs still converge to those of the dense pencil (brute force) while
    the filter applies fewer band-degrees than the fixed-degree loop."""
    pb, ops, lp = mid_run
    H = dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D)
    S = dense.overlap(pb.npw, pb.P, pb.Q)
    exact = dense.eig_pencil(H, S)[0]
    tol = 1e-8
    lam, X, res, hist = matfree.chebfsi(ops, pb.X0, pb.cfg.m, 12, lp, lock_tol=tol)
    done = res <= 2 * tol  # locked bands hover just below tol
    assert done[:20].all()
    assert np.all(np.abs(lam[done] - exact[:pb.cfg.nb][done]) <= 1e-12 * np.maximum(np.abs(exact[:pb.cfg.nb][done]), 1))
    # bands still far from tol got the full degree every time: same residuals as without locking
    res_full = matfree.chebfsi(ops, pb.X0, pb.cfg.m, 12, lp)[2]
    slow = res_full > 100 * tol
    assert slow.sum() >= 8 and np.allclose(res[slow], res_full[slow], rtol=1e-3)
    work = sum(int(h["degrees"].sum()) for h in hist)
    assert work < 0.8 * pb.cfg.nb * pb.cfg.m * len(hist)
    assert any((h["degrees"] == 0).any() for h in hist)  # some bands were locked


# ---- capacitance solve by preconditioned iterative refinement (Sec. 5.1) ---------------------------------------
@pytest.fixture(scope="module")
def cap_mid():
    pb = wl.make_problem("mid_paw")
    C = np.diag(1.0 / pb.Q).astype(complex) + pb.P.conj().T @ pb.P
    return pb, C, matfree.atom_blocks(pb.proj_off)


def test_capacitance_refinement_converges_to_direct_solve(cap_mid):
    pb, C, blocks = cap_mid
    b = np.random.default_rng(3).normal(size=(pb.nproj, 5)) + 1j * np.random.default_rng(4).normal(size=(pb.nproj, 5))
    q, k, hist = matfree.capacitance_refine(C, blocks, b)
    direct = scipy.linalg.cho_solve(scipy.linalg.cho_factor(C), b)
    assert np.linalg.norm(q - direct) <= 1e-13 * np.linalg.norm(direct)
    assert 1 <= k <= 60 and hist[-1] <= 1e-15


def test_capacitance_refinement_contraction(cap_mid):
    """The error shrinks by the spectral radius of I - M^-1 C per correction (the iteration's algebra: a wrong
    sign in the update diverges), and an exactly block-diagonal C is solved by the preconditioner alone."""
    pb, C, blocks = cap_mid
    Minv = matfree.block_preconditioner(C, blocks)
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(pb.nproj) - Minv @ C)))
    assert 0 < rho < 1
    b = np.random.default_rng(5).normal(size=pb.nproj) + 0j
    exact = np.linalg.solve(C, b)
    errs = [np.linalg.norm(matfree.capacitance_refine(C, blocks, b, iters=k)[0] - exact) for k in range(0, 9)]
    ratios = np.array(errs[5:]) / np.array(errs[4:-1])
    assert np.all(ratios <= rho * 1.05) and np.all(ratios >= 0.2 * rho)
    Cb = np.zeros_like(C)
    for s, n in blocks:
        Cb[s:s + n, s:s + n] = C[s:s + n, s:s + n]
    q, k, hist = matfree.capacitance_refine(Cb, blocks, b)
    assert k == 0 and np.allclose(q, np.linalg.solve(Cb, b), atol=1e-14 * np.linalg.norm(q))


# ---- LOBPCG, the block method the paper compares with (Sec. 2.3) -----------------------------------------------
from oracle import lobpcg as lobpcg_oracle  # noqa: E402


def test_tpa_preconditioner_function():
    """K(0) = 1, K(1) = 65/81, decreasing, K(x) 2x -> 1 for large x (damps as the inverse kinetic energy)."""
    K = lobpcg_oracle.tpa
    assert K(0.0) == 1.0 and abs(K(1.0) - 65.0 / 81.0) < 1e-15
    x = np.linspace(0, 50, 1001)
    assert np.all(np.diff(K(x)) < 0)
    assert abs(K(1e6) * 2e6 - 1.0) < 1e-5


@pytest.mark.parametrize("name", ["nc16", "tiny_paw"])
def test_lobpcg_converges_to_dense_eigenpairs(name):
    pb = wl.make_problem(name)
    ops = matfree.Operators.from_problem(pb)
    H = dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D)
    S = dense.overlap(pb.npw, pb.P, pb.Q)
    exact = dense.eig_pencil(H, S)[0]
    nw = pb.cfg.nb - pb.cfg.nb // 8
    lam, X, res, hist = lobpcg_oracle.lobpcg(ops, pb.X0, 40)
    assert np.all(np.abs(lam[:nw] - exact[:nw]) <= 1e-10 * np.maximum(np.abs(exact[:nw]), 1.0))
    assert np.all(res[:nw] <= 2e-8)
    # Courant-Fischer: X lies in every Rayleigh-Ritz space, so no Ritz value ever increases
    for a, b in zip(hist[:-1], hist[1:]):
        assert np.all(b["ritz"] <= a["ritz"] + 1e-10)
    # X is S-orthonormal
    assert np.allclose(X.conj().T @ (S @ X), np.eye(X.shape[1]), atol=1e-9)


def test_lobpcg_preconditioner_accelerates():
    pb = wl.make_problem("tiny_paw")
    ops = matfree.Operators.from_problem(pb)
    nw = pb.cfg.nb - pb.cfg.nb // 8

    def iters_to(precond):
        hist = lobpcg_oracle.lobpcg(ops, pb.X0, 60, precond=precond)[3]
        return next(h["it"] for h in hist[1:] if h["resid"][:nw].max() <= 1e-6)
    assert iters_to(True) < iters_to(False)


# ---- Gamma point: real wavefunctions on the half sphere (Sec. 2.1) -----------------------------------------------
from oracle import gamma as gamma_oracle  # noqa: E402


@pytest.fixture(scope="module")
def gam():
    gp = wl.make_gamma_problem("tiny_paw")
    return gp, gamma_oracle.GammaOperators.from_problem(gp)


def test_gamma_projectors_real_in_real_space(gam):
    """With the (-i)^l factor, P(-G) = conj P(G): every projector is a real function on the grid."""
    gp, _ = gam
    n = gp.cfg.n
    for j in range(gp.nproj):
        box = np.zeros((n, n, n), complex)
        box[tuple((gp.full.gidx % n).T)] = gp.full.P[:, j]
        real = dense.naive_dft3(box, +1) if n <= 12 else np.fft.ifftn(box) * n**3
        assert np.abs(real.imag).max() <= 1e-12 * np.abs(real).max()


def test_gamma_expand_contract(gam):
    gp, ops = gam
    gm = ops.map
    Y = gp.X0
    assert np.allclose(gm.expand(Y), gp.full.X0, atol=1e-15)  # the generator's expansion agrees
    assert np.allclose(gm.contract(gm.expand(Y)), Y, atol=1e-14)
    # inner products: Re <y, z> on the half sphere = <expand y, expand z> on the whole sphere
    Z = np.random.default_rng(2).normal(size=Y.shape) + 0j
    Z[gm.zero] = Z[gm.zero].real
    assert np.allclose(np.real(Y.conj().T @ Z), gm.expand(Y).conj().T @ gm.expand(Z), atol=1e-11)
    # expanded vectors are real functions on the grid
    n = gp.cfg.n
    box = np.zeros((n, n, n), complex)
    box[tuple((gp.full.gidx % n).T)] = gm.expand(Y[:, 0])[:, 0]
    assert np.abs(np.fft.ifftn(box).imag).max() <= 1e-14


def test_gamma_spectrum_equals_complex_spectrum(gam):
    """H restricted to real functions is the real symmetric matrix of the full Hermitian H: same spectrum
    (the complex problem with real-space-real projectors is the complexification of the real one)."""
    gp, ops = gam
    Hr = gamma_oracle.dense_real(ops, "H")
    Sr = gamma_oracle.dense_real(ops, "S")
    assert np.allclose(Hr, Hr.T, atol=1e-12) and np.allclose(Sr, Sr.T, atol=1e-13)
    H = dense.hamiltonian(gp.full.gidx, gp.full.kin, gp.full.V, gp.full.P, gp.full.D)
    S = dense.overlap(gp.full.npw, gp.full.P, gp.full.Q)
    lam_c = dense.eig_pencil(H, S)[0]
    lam_r = scipy.linalg.eigh(Hr, Sr, eigvals_only=True)
    assert Hr.shape[0] == gp.full.npw
    assert np.allclose(lam_r, lam_c, atol=1e-11)


def test_gamma_outer_loop_converges(gam):
    gp, ops = gam
    H = dense.hamiltonian(gp.full.gidx, gp.full.kin, gp.full.V, gp.full.P, gp.full.D)
    S = dense.overlap(gp.full.npw, gp.full.P, gp.full.Q)
    exact = dense.eig_pencil(H, S)[0]
    lp = matfree.lanczos_upper_bound(ops.full, gp.full.v0, 10)[0]
    lam, X, res, hist = gamma_oracle.chebfsi(ops, gp.X0, gp.cfg.m, 30, lp)
    nw = gp.cfg.nb - gp.cfg.nb // 8
    assert np.all(np.abs(lam[:nw] - exact[:nw]) <= 1e-10 * np.maximum(np.abs(exact[:nw]), 1.0))
    assert np.abs(X[ops.map.zero].imag).max() <= 1e-12 * np.abs(X).max()  # still real functions
