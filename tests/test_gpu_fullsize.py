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
    pb = wl.make_problem("paw64", ndir=1)
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
    # central differences of the GPU FP64 forward along one V direction (one Richardson step)
    E = torch.from_numpy(pb.dV[0])
    V = torch.from_numpy(pb.V)

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
    p64.set_potential(V)
    an = float(torch.sum(dV.cpu() * E))
    assert abs(fd - an) <= 1e-5 * abs(fd), (fd, an)
    # complex64 adjoint against the FP64 one
    pm = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    _, dXm, dVm, dDm = pm.filter_rr_backward(cf.to_device_block(pb.X0, torch.complex64), m, c, r, w, 3)
    ev = _rel(dVm.cpu().numpy(), dV.cpu().numpy())
    ed = _rel(dDm.cpu().numpy(), dD.cpu().numpy())
    print(f"paw64 mixed adjoint vs FP64: dV {ev:.2e} dD {ed:.2e}")
    assert ev < 1e-3 and ed < 1e-3


@pytest.mark.parametrize("name", ["paw96", "paw128"])
def test_large_shapes_mixed(name):
    pb = wl.make_problem(name)
    print(f"[case] {pb.cfg.name} npw={pb.npw} nb={pb.cfg.nb} nproj={pb.nproj}", flush=True)
    plan = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    print("[step] plan ready", flush=True)
    c, r, lp = _interval(plan, pb, torch.complex64)
    X = cf.to_device_block(pb.X0, torch.complex64)
    plan.filter(X, pb.cfg.m, c, r)
    torch.cuda.synchronize()
    print("[step] filter done", flush=True)
    cols = [0, pb.cfg.nb // 2, pb.cfg.nb - 1]
    _sampled_filter_check(pb, X, pb.cfg.m, c, r, cols, 2e-4)
    ritz, res = plan.rayleigh_ritz(X)
    ritz = ritz.cpu().numpy()
    assert np.all(np.diff(ritz) >= 0) and np.all(np.isfinite(res.cpu().numpy()))
