"""Parity of the hand-written adjoint (cheb_filter_rr_backward) with the FP64 oracle adjoint, which is itself
pinned by finite differences; plus the autograd wrapper and checkpoint-interval independence."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import dense, grad, matfree  # noqa: E402
from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402
from paper_1406_4350_amd.autograd import ChebFilterRR  # noqa: E402


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _setup(name, nb, nk, m):
    pb = wl.make_problem(wl.config(name).replace(nb=nb))
    ops = matfree.Operators.from_problem(pb)
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lm = float(np.max(matfree.rayleigh_quotients(ops, pb.X0)))
    c, r = 0.5 * (lp + lm), 0.5 * (lp - lm)
    w = np.random.default_rng(3).uniform(0, 1, nk)
    return pb, ops, c, r, w, m


CASES = [("tiny_paw", 10, 6, 3), ("mid_nc", 20, 9, 4), ("mid_paw", 16, 8, 5), ("nc16", 16, 8, 4)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-nb{c[1]}-m{c[3]}")
def case(request):
    name, nb, nk, m = request.param
    pb, ops, c, r, w, m = _setup(name, nb, nk, m)
    print(f"[case] {pb.cfg.name} nb={nb} nk={nk} m={m}", flush=True)
    ref = grad.filter_rr_grad(ops, pb.X0, m, c, r, w, pb.D)
    return pb, ops, c, r, w, m, ref


@pytest.mark.parametrize("ckpt", [1, 2, 3])
def test_backward_fp64_matches_oracle(case, ckpt):
    pb, ops, c, r, w, m, (L, lam, dX, dV, dD) = case
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    X0 = cf.to_device_block(pb.X0, torch.complex128)
    ritz, gX, gV, gD = plan.filter_rr_backward(X0, m, c, r, w, ckpt)
    ritz = ritz.cpu().numpy()
    assert np.all(np.abs(ritz - lam) <= 1e-10 * np.maximum(np.abs(lam), 1.0))
    assert _rel(cf.to_host_block(gX), dX) < 1e-8
    assert _rel(gV.cpu().numpy(), dV) < 1e-8
    if pb.nproj:
        assert _rel(gD.cpu().numpy(), dD) < 1e-8


def test_backward_mixed(case):
    pb, ops, c, r, w, m, (L, lam, dX, dV, dD) = case
    plan = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    X0 = cf.to_device_block(pb.X0, torch.complex64)
    ritz, gX, gV, gD = plan.filter_rr_backward(X0, m, c, r, w, 3)
    ev, ex = _rel(gV.cpu().numpy(), dV), _rel(cf.to_host_block(gX), dX)
    print(f"mixed adjoint vs FP64 oracle: dV {ev:.2e}  dX {ex:.2e}")
    assert ev < 1e-3 and ex < 1e-3


def test_autograd_wrapper():
    pb, ops, c, r, w, m = _setup("tiny_paw", 10, 6, 3)
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    X0 = cf.to_device_block(pb.X0, torch.complex128).requires_grad_(True)
    V = torch.from_numpy(pb.V.copy()).cuda().requires_grad_(True)
    D = torch.from_numpy(pb.D_packed).cuda().requires_grad_(True)
    ritz = ChebFilterRR.apply(X0, V, D, plan, m, c, r, 2)
    L = (ritz[:6] * torch.from_numpy(w).cuda()).sum()
    gX, gV, gD = torch.autograd.grad(L, (X0, V, D))
    Lr, lam, dX, dV, dD = grad.filter_rr_grad(ops, pb.X0, m, c, r, w, pb.D)
    assert abs(L.item() - Lr) < 1e-10 * max(1.0, abs(Lr))
    assert _rel(cf.to_host_block(gX), 2.0 * dX) < 1e-8
    assert _rel(gV.cpu().numpy(), dV) < 1e-8
    assert _rel(gD.cpu().numpy(), dD) < 1e-8


def test_backward_argument_errors():
    pb, ops, c, r, w, m = _setup("tiny_paw", 10, 6, 3)
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    X0 = cf.to_device_block(pb.X0, torch.complex128)
    for bad in (dict(m=0), dict(ckpt_every=0), dict(r=-1.0)):
        kw = dict(m=m, c=c, r=r, w=w, ckpt_every=2)
        kw.update(bad)
        with pytest.raises(cf.ChebError) as e:
            plan.filter_rr_backward(X0, **kw)
        assert e.value.status == cf.CHEB_ERR_ARG
    with pytest.raises(cf.ChebError):
        plan.filter_rr_backward(X0, m, c, r, np.ones(11), 2)  # nk > nb


@pytest.mark.parametrize("n,radius", [(96, 9), (128, 10)])
def test_backward_large_boxes(n, radius):
    """The adjoint on the 96^3 and 128^3 boxes, where the cross density of dL/dV(r) is taken in its polarisation
    form (two single-field densities), against the FP64 oracle adjoint; mixed precision against the FP64 one."""
    cfg = wl.SMALL["tiny_paw"].replace(name=f"adj{n}", n=n, radius=radius, nb=8, seed_index=300 + n)
    pb = wl.make_problem(cfg)
    ops = matfree.Operators.from_problem(pb)
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lm = float(np.max(matfree.rayleigh_quotients(ops, pb.X0)))
    c, r = 0.5 * (lp + lm), 0.5 * (lp - lm)
    m, nk = 3, 5
    w = np.random.default_rng(7).uniform(0, 1, nk)
    print(f"[case] n={n} R={radius} npw={pb.npw} nb=8 m={m}", flush=True)
    L, lam, dX, dV, dD = grad.filter_rr_grad(ops, pb.X0, m, c, r, w, pb.D)
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    ritz, gX, gV, gD = plan.filter_rr_backward(cf.to_device_block(pb.X0, torch.complex128), m, c, r, w, 2)
    assert np.all(np.abs(ritz.cpu().numpy() - lam) <= 1e-10 * np.maximum(np.abs(lam), 1.0))
    assert _rel(cf.to_host_block(gX), dX) < 1e-8
    assert _rel(gV.cpu().numpy(), dV) < 1e-8
    assert _rel(gD.cpu().numpy(), dD) < 1e-8
    pm = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    _, mX, mV, mD = pm.filter_rr_backward(cf.to_device_block(pb.X0, torch.complex64), m, c, r, w, 2)
    ev = _rel(mV.cpu().numpy(), dV)
    print(f"[check] mixed adjoint vs FP64 oracle: dV {ev:.2e}", flush=True)
    assert ev < 1e-3
