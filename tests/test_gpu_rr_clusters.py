"""Rayleigh-Ritz with strongly coupled clusters (the subspace eigenproblem of Sec. 3).

Blocks whose columns are the exact eigenvectors of the pencil, mixed by unitary rotations inside groups of
neighbouring eigenvalues (pairs turned by 45 degrees, so that the first-order correction is unbounded), are
solved by the warm-started refinement with exact cluster solves, without the library eigensolver, to the
dense pencil's eigenvalues (1e-10 max(|lambda|, 1)) and S-orthonormal Ritz vectors. A group larger than the
cluster limit (48) goes to the library eigensolver with the same result.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import dense  # noqa: E402
from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402


@pytest.fixture(scope="module", params=["mid_paw", "mid_nc"], ids=str)
def case(request):
    pb = wl.make_problem(request.param)
    H = dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D)
    S = dense.overlap(pb.npw, pb.P, pb.Q)
    lam, U = dense.eig_pencil(H, S)
    print(f"[case] {pb.cfg.name} npw={pb.npw} nb={pb.cfg.nb}", flush=True)
    return pb, H, S, lam, U, cf.plan_from_problem(pb, cf.CHEB_FP64)


def _mixed(U, groups, seed):
    rng = np.random.default_rng(seed)
    X = U.copy()
    for g in groups:
        if len(g) == 2:
            ph = np.exp(2j * np.pi * rng.uniform())
            R = np.array([[1.0, -ph.conjugate()], [ph, 1.0]]) / np.sqrt(2.0)
        else:
            R, _ = np.linalg.qr(rng.standard_normal((len(g), len(g))) + 1j * rng.standard_normal((len(g), len(g))))
        X[:, g] = U[:, g] @ R
    return X * rng.uniform(0.5, 2.0, X.shape[1])[None, :]


def _check(pb, S, lam, Xd, ritz):
    nb = pb.cfg.nb
    ritz = ritz.cpu().numpy()
    assert np.all(np.abs(ritz - lam[:nb]) <= 1e-10 * np.maximum(np.abs(lam[:nb]), 1.0))
    Ug = cf.to_host_block(Xd)
    assert np.allclose(Ug.conj().T @ (S @ Ug), np.eye(nb), atol=1e-9)


def test_clusters_refined(case):
    pb, H, S, lam, U, plan = case
    nb = pb.cfg.nb
    sizes, groups, i = [2, 3, 2, 4, 1, 2, 5], [], 0
    while i < nb:
        k = min(sizes[len(groups) % len(sizes)], nb - i)
        if k > 1:
            groups.append(list(range(i, i + k)))
        i += k
    X = _mixed(U[:, :nb], groups, 7)
    plan.set_rr_refine(True)
    before = plan.rr_stats()
    Xd = cf.to_device_block(X, torch.complex128)
    ritz, res = plan.rayleigh_ritz(Xd)
    after = plan.rr_stats()
    assert after == (before[0] + 1, before[1]), (before, after)  # refined, no library call
    _check(pb, S, lam, Xd, ritz)
    assert res.cpu().numpy().max() <= 1e-8 * max(1.0, float(np.abs(lam[:nb]).max()))


def test_cluster_over_limit_goes_to_library(case):
    pb, H, S, lam, U, plan = case
    nb = pb.cfg.nb
    if nb < 50:
        pytest.skip("block smaller than the cluster limit")
    X = _mixed(U[:, :nb], [list(range(0, 50))], 11)
    plan.set_rr_refine(True)
    before = plan.rr_stats()
    Xd = cf.to_device_block(X, torch.complex128)
    ritz, _ = plan.rayleigh_ritz(Xd)
    after = plan.rr_stats()
    assert after == (before[0], before[1] + 1), (before, after)
    _check(pb, S, lam, Xd, ritz)
