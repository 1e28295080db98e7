"""Full-size workloads on the GPU: the paw48 block exactly as bench.py times it, the differentiation form at
paw64, and the large paw96 / paw128 shapes. Outputs the oracle can compute one by one (single bands of the
filter, which acts on bands independently) are compared directly; the rest through properties that hold at
any size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import matfree  # noqa: E402
from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _interval(plan, pb, dtype):
    lp = plan.upper_bound(torch.from_numpy(pb.v0), 10)
    lm = float(plan.rayleigh_quotients(cf.to_device_block(pb.X0, dtype)).max())
    return 0.5 * (lp + lm), 0.5 * (lp - lm), lp


def _sampled_filter_check(pb, Xd, m, c, r, cols, tol):
    print(f"[check] oracle filter on bands {cols}", flush=True)
    ops = matfree.Operators.from_problem(pb, band_chunk=8)
    ref = matfree.chebyshev_filter(ops, pb.X0[:, cols], m, c, r)
    got = cf.to_host_block(Xd[cols])
    for k in range(len(cols)):
        assert _rel(got[:, k], ref[:, k]) < tol, (cols[k], _rel(got[:, k], ref[:, k]))


def test_paw48_bench_block():
    pb = wl.make_problem("paw48")
    print(f"[case] paw48 npw={pb.npw} nb={pb.cfg.nb}", flush=True)
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    c, r, lp = _interval(plan, pb, torch.complex128)
    X = cf.to_device_block(pb.X0, torch.complex128)
    plan.filter(X, pb.cfg.m, c, r)
    cols = [0, 97, 181, 255]
    _sampled_filter_check(pb, X, pb.cfg.m, c, r, cols, 1e-11)
    Y = cf.to_host_block(X)
    ritz, res = plan.rayleigh_ritz(X)
    lam, _, res_o = matfree.rayleigh_ritz(matfree.Operators.from_problem(pb), Y)
    ritz = ritz.cpu().numpy()
    assert np.all(np.abs(ritz - lam) <= 1e-10 * np.maximum(np.abs(lam), 1.0))
    # mixed path, same block: complex64 rounding amplified by the degree-8 recurrence
    pm = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    Xm = cf.to_device_block(pb.X0, torch.complex64)
    pm.filter(Xm, pb.cfg.m, c, r)
    _sampled_filter_check(pb, Xm, pb.cfg.m, c, r, cols, 1e-4)


def test_paw48_filter_degrees():
    """Locking at the bench shape: per-band degrees 0..m in scrambled order; sampled bands of each degree
    against the oracle filter of that degree on that band alone."""
    pb = wl.make_problem("paw48")
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    c, r, _ = _interval(plan, pb, torch.complex128)
    m = pb.cfg.m
    deg = np.random.default_rng(5).integers(0, m + 1, pb.cfg.nb).astype(np.int32)
    X = cf.to_device_block(pb.X0, torch.complex128)
    plan.filter_degrees(X, deg, c, r)
    ops = matfree.Operators.from_problem(pb, band_chunk=8)
    for d in (0, 1, 4, m - 1, m):
        cols = list(np.nonzero(deg == d)[0][:2])
        print(f"[check] degree {d} bands {cols}", flush=True)
        ref = matfree.chebyshev_filter(ops, pb.X0[:, cols], d, c, r)
        got = cf.to_host_block(X[cols])
        for k in range(len(cols)):
            assert _rel(got[:, k], ref[:, k]) < 1e-11


def test_paw64_backward_full():
    pb = wl.make_problem("paw64", ndir=8)
    print(f"[case] paw64 npw={pb.npw} nb={pb.cfg.nb} nk={pb.cfg.nk}", flush=True)
    p64 = cf.plan_from_problem(pb, cf.CHEB_FP64)
    c, r, lp = _interval(p64, pb, torch.complex128)
    m, nk = pb.cfg.m, pb.cfg.nk
    w = pb.w
    X0 = cf.to_device_block(pb.X0, torch.complex128)
    ritz, dX, dV, dD = p64.filter_rr_backward(X0, m, c, r, w, 3)
    # L depends on X0 through its span only
    inv = torch.linalg.matrix_norm(X0.conj() @ dX.T) / (torch.linalg.matrix_norm(X0) * torch.linalg.matrix_norm(dX))
    assert inv.item() < 1e-9
    # central differences (h = 1e-4, one Richardson step) of the GPU FP64 forward along the 8 random V(r)
    # directions of the differentiation form
    V = torch.from_numpy(pb.V)
    for k in range(pb.dV.shape[0]):
        E = torch.from_numpy(pb.dV[k])

        def loss(t):
            p64.set_potential(V + t * E)
            Y = X0.clone()
            p64.filter(Y, m, c, r)
            lam = p64.rayleigh_ritz(Y, with_residuals=False)[0].cpu().numpy()
            return float(np.dot(w, lam[:nk]))
        h = 1e-4
        d1 = (loss(h) - loss(-h)) / (2 * h)
        d2 = (loss(h / 2) - loss(-h / 2)) / h
        fd = (4 * d2 - d1) / 3
        an = float(torch.sum(dV.cpu() * E))
        print(f"[fd] direction {k}: finite difference {fd:.10e}, adjoint {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-5 * abs(fd), (k, fd, an)
    p64.set_potential(V)
    # complex64 adjoint against the FP64 one
    pm = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    _, dXm, dVm, dDm = pm.filter_rr_backward(cf.to_device_block(pb.X0, torch.complex64), m, c, r, w, 3)
    ev = _rel(dVm.cpu().numpy(), dV.cpu().numpy())
    ed = _rel(dDm.cpu().numpy(), dD.cpu().numpy())
    print(f"paw64 mixed adjoint vs FP64: dV {ev:.2e} dD {ed:.2e}")
    assert ev < 1e-3 and ed < 1e-3


@pytest.fixture(scope="module", params=["paw96", "paw128"])
def large(request):
    """A large workload and the oracle's operators on it (the capacitance factorisation is built once)."""
    pb = wl.make_problem(request.param)
    print(f"[case] {pb.cfg.name} npw={pb.npw} nb={pb.cfg.nb} nproj={pb.nproj}", flush=True)
    return pb, matfree.Operators.from_problem(pb, band_chunk=8)


def _sampled_against(ops, pb, Xd, m, c, r, cols, tol):
    print(f"[check] oracle filter on bands {cols}", flush=True)
    ref = matfree.chebyshev_filter(ops, pb.X0[:, cols], m, c, r)
    got = cf.to_host_block(Xd[cols])
    for k in range(len(cols)):
        assert _rel(got[:, k], ref[:, k]) < tol, (cols[k], _rel(got[:, k], ref[:, k]))


def _rotated_block_checks(plan, X, ritz, res, cols, tol):
    """Properties of a Rayleigh-Ritz result that hold at any size, on sampled columns: ascending Ritz values,
    S-orthonormal columns, Rayleigh quotients equal to the Ritz values, reported residuals equal to
    ||H u - lambda S u|| recomputed from the rotated vectors."""
    ritz, res = ritz.cpu().numpy(), res.cpu().numpy()
    assert np.all(np.diff(ritz) >= 0) and np.all(np.isfinite(res))
    U = X[cols].contiguous()
    HU, SU = plan.apply_H(U), plan.apply_S(U)
    # u_i^H S u_j summed in FP64 (a complex64 product sums tens of thousands of terms in FP32)
    G = (U.to(torch.complex128).conj() @ SU.to(torch.complex128).T).cpu().numpy()
    assert np.abs(G - np.eye(len(cols))).max() < tol
    rq = plan.rayleigh_quotients(U).cpu().numpy()
    assert np.all(np.abs(rq - ritz[cols]) <= tol * np.maximum(np.abs(ritz[cols]), 1.0))
    lam = torch.from_numpy(ritz[cols]).to(U.device)
    r2 = torch.linalg.vector_norm(HU - SU * lam[:, None], dim=1).cpu().numpy()
    assert np.allclose(r2, res[cols], rtol=1e-3, atol=100 * tol)


def test_large_shapes_fp64(large):
    """FP64 plans at the 96^3 and 128^3 boxes: one H application and one degree-m filter of the full block
    against the oracle on sampled bands, then Rayleigh-Ritz of the whole block checked by its properties."""
    pb, ops = large
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    print("[step] plan ready", flush=True)
    c, r, lp = _interval(plan, pb, torch.complex128)
    X = cf.to_device_block(pb.X0, torch.complex128)
    cols = [0, 1, pb.cfg.nb // 2 + 3, pb.cfg.nb - 1]
    HX = plan.apply_H(X[cols].contiguous())
    ref = ops.apply_H(pb.X0[:, cols])
    assert _rel(cf.to_host_block(HX), ref) < 1e-12
    plan.filter(X, pb.cfg.m, c, r)
    torch.cuda.synchronize()
    print("[step] filter done", flush=True)
    _sampled_against(ops, pb, X, pb.cfg.m, c, r, cols, 1e-11)
    ritz, res = plan.rayleigh_ritz(X)
    print("[step] rayleigh-ritz done", flush=True)
    _rotated_block_checks(plan, X, ritz, res, cols, 1e-10)
    plan.close()


def test_large_shapes_mixed(large):
    pb, ops = large
    plan = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    print("[step] plan ready", flush=True)
    c, r, lp = _interval(plan, pb, torch.complex64)
    X = cf.to_device_block(pb.X0, torch.complex64)
    plan.filter(X, pb.cfg.m, c, r)
    torch.cuda.synchronize()
    print("[step] filter done", flush=True)
    cols = [0, pb.cfg.nb // 2, pb.cfg.nb - 1]
    _sampled_against(ops, pb, X, pb.cfg.m, c, r, cols, 2e-4)
    ritz, res = plan.rayleigh_ritz(X)
    # complex64 vectors: S-orthonormality and quotients hold to float32 rounding
    _rotated_block_checks(plan, X, ritz, res, cols, 2e-5)
    plan.close()
