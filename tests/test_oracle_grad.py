"""Pins of the oracle's adjoint (filter + Rayleigh-Ritz) against central finite differences of the forward,
span invariance, and Hellmann-Feynman at an exact invariant subspace."""
import numpy as np
import pytest

from oracle import dense, grad, matfree
from paper_1406_4350_amd import workload as wl


@pytest.fixture(scope="module", params=["tiny_paw", "nc"])
def setup(request):
    if request.param == "tiny_paw":
        pb = wl.make_problem(wl.SMALL["tiny_paw"].replace(nb=10), ndir=2)
    else:
        pb = wl.make_problem(wl.CONFIGS["nc16"].replace(nb=10), ndir=2)
    ops = matfree.Operators.from_problem(pb)
    lam = dense.eig_pencil(dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D), dense.overlap(pb.npw, pb.P, pb.Q))[0]
    c, r = 0.5 * (lam[-1] + lam[12]), 0.5 * (lam[-1] - lam[12]) + 0.1
    w = np.random.default_rng(5).uniform(0, 1, 6)
    m = 3
    L, ritz, dX, dV, dD = grad.filter_rr_grad(ops, pb.X0, m, c, r, w, pb.D)
    return pb, ops, c, r, w, m, L, dX, dV, dD


def _ops_with(pb, V=None, D=None):
    return matfree.Operators(pb.gidx, pb.kin, pb.V if V is None else V, pb.P, pb.D if D is None else D, pb.Q)


def _fd(f, h):
    """Central difference with one Richardson step: (4 D(h/2) - D(h)) / 3, error O(h^4)."""
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_fd_potential(setup):
    pb, ops, c, r, w, m, L, dX, dV, dD = setup
    h = 1e-4
    for k in range(pb.dV.shape[0]):
        E = pb.dV[k]
        fd = _fd(lambda t: grad.loss(_ops_with(pb, V=pb.V + t * E), pb.X0, m, c, r, w), h)
        an = float(np.sum(dV * E))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (fd, an)


def test_fd_D(setup):
    pb, ops, c, r, w, m, L, dX, dV, dD = setup
    if pb.nproj == 0:
        pytest.skip("no projectors")
    rng = np.random.default_rng(11)
    E = []
    for d in pb.D:
        e = rng.normal(size=d.shape)
        E.append(e + e.T)
    Ep = np.concatenate([e.ravel() for e in E])
    h = 1e-4
    fd = _fd(lambda t: grad.loss(_ops_with(pb, D=[d + t * e for d, e in zip(pb.D, E)]), pb.X0, m, c, r, w), h)
    an = float(np.dot(dD, Ep))
    assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (fd, an)


def test_fd_start_block_and_invariance(setup):
    pb, ops, c, r, w, m, L, dX, dV, dD = setup
    rng = np.random.default_rng(12)
    E = rng.normal(size=pb.X0.shape) + 1j * rng.normal(size=pb.X0.shape)
    h = 1e-4
    fd = _fd(lambda t: grad.loss(ops, pb.X0 + t * E, m, c, r, w), h)
    an = 2.0 * float(np.real(np.vdot(dX, E)))
    assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (fd, an)
    # L depends on X0 only through its span: X0^H dL/dX0 = 0
    assert np.linalg.norm(pb.X0.conj().T @ dX) <= 1e-9 * np.linalg.norm(pb.X0) * np.linalg.norm(dX)


def test_hellmann_feynman_at_invariant_subspace():
    """X0 spanning exact eigenvectors: residuals vanish, so dL/dX0 = 0 and dL/dV_j = n^-3 sum w |u_i(r_j)|^2,
    whose grid sum is sum_i w_i ||u_i||^2 (Parseval)."""
    pb = wl.make_problem("tiny_paw")
    ops = matfree.Operators.from_problem(pb)
    H = dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D)
    S = dense.overlap(pb.npw, pb.P, pb.Q)
    lam, Vec = dense.eig_pencil(H, S)
    M = np.random.default_rng(2).normal(size=(8, 8))
    X0 = Vec[:, :8] @ M
    w = np.linspace(0.2, 1.0, 5)
    c, r = 0.5 * (lam[-1] + lam[10]), 0.5 * (lam[-1] - lam[10])
    L, ritz, dX, dV, dD = grad.filter_rr_grad(ops, X0, 4, c, r, w, pb.D)
    assert np.allclose(ritz, lam[:8], atol=1e-10)
    assert np.linalg.norm(dX) < 1e-8 * np.linalg.norm(X0)
    U = Vec[:, :5]
    hf = np.einsum("b,bxyz->xyz", w, np.abs(grad.real_space(ops, U)) ** 2) / pb.cfg.n**3
    assert np.allclose(dV, hf, atol=1e-9 * np.abs(hf).max())
    assert abs(dV.sum() - np.sum(w * np.sum(np.abs(U) ** 2, axis=0))) < 1e-9


def test_planted_factor_error_is_caught(setup, monkeypatch):
    """Dropping the factor 2 of the filter's V term must break the finite-difference pin."""
    pb, ops, c, r, w, m, L, dX, dV, dD = setup
    orig = grad.real_space
    calls = {"n": 0}

    def halve_filter_terms(o, psi):  # the first real_space call is the Hellmann-Feynman one
        calls["n"] += 1
        out = orig(o, psi)
        return out if calls["n"] == 1 else out * np.sqrt(0.5)
    monkeypatch.setattr(grad, "real_space", halve_filter_terms)
    _, _, _, dV_bad, _ = grad.filter_rr_grad(ops, pb.X0, m, c, r, w, pb.D)
    E = pb.dV[0]
    h = 1e-4
    fd = (grad.loss(_ops_with(pb, V=pb.V + h * E), pb.X0, m, c, r, w)
          - grad.loss(_ops_with(pb, V=pb.V - h * E), pb.X0, m, c, r, w)) / (2 * h)
    assert abs(fd - float(np.sum(dV_bad * E))) > 1e-4 * abs(fd)
