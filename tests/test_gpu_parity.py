"""Parity of the HIP path (through the C ABI) with the FP64 oracle on identical seeded inputs.

FP64 plans: operator applications to 1e-12 relative, the filter to 1e-11 relative (its output is a
degree-m polynomial; rounding grows with the recurrence), Ritz values to |d lambda| <= 1e-10 max(|lambda|, 1)
(the stated FP64 target). Mixed plans (complex64 bands, FP32-MFMA GEMMs) are held to bounds derived from
float32 rounding: 2e-5 relative per operator application.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import matfree  # noqa: E402
from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402
from paper_1406_4350_amd.driver import chebfsi  # noqa: E402

CASES = ["nc16", "tiny_paw", "mid_paw", "mid_nc"]


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module", params=CASES, ids=str)
def case(request):
    pb = wl.make_problem(request.param)
    print(f"[case] {pb.cfg.name} npw={pb.npw} nproj={pb.nproj} nb={pb.cfg.nb}", flush=True)
    ops = matfree.Operators.from_problem(pb)
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    return pb, ops, plan


def test_apply_operators(case):
    pb, ops, plan = case
    X = pb.X0
    Xd = cf.to_device_block(X, torch.complex128)
    assert _rel(cf.to_host_block(plan.apply_H(Xd)), ops.apply_H(X)) < 1e-12
    assert _rel(cf.to_host_block(plan.apply_S(Xd)), ops.apply_S(X)) < 1e-12
    assert _rel(cf.to_host_block(plan.apply_Sinv(Xd)), ops.apply_Sinv(X)) < 1e-12


@pytest.mark.parametrize("m", [0, 1, 2, 5])
def test_filter(case, m):
    pb, ops, plan = case
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lm = float(np.max(matfree.rayleigh_quotients(ops, pb.X0)))
    c, r = 0.5 * (lp + lm), 0.5 * (lp - lm)
    Xd = cf.to_device_block(pb.X0, torch.complex128)
    plan.filter(Xd, m, c, r)
    ref = matfree.chebyshev_filter(ops, pb.X0, m, c, r)
    assert _rel(cf.to_host_block(Xd), ref) < 1e-11


def test_rayleigh_ritz(case):
    pb, ops, plan = case
    Y = matfree.chebyshev_filter(ops, pb.X0, 3, 1.0, 2.0)
    lam, U, res = matfree.rayleigh_ritz(ops, Y)
    Yd = cf.to_device_block(Y, torch.complex128)
    ritz, rd = plan.rayleigh_ritz(Yd)
    ritz = ritz.cpu().numpy()
    assert np.all(np.abs(ritz - lam) <= 1e-10 * np.maximum(np.abs(lam), 1.0))
    assert np.allclose(rd.cpu().numpy(), res, rtol=1e-6, atol=1e-9)
    # rotated block is S-orthonormal
    Ug = cf.to_host_block(Yd)
    SU = ops.apply_S(Ug)
    assert np.allclose(Ug.conj().T @ SU, np.eye(Ug.shape[1]), atol=1e-9)
    # and spans the oracle's Ritz subspaces: eigenvectors are compared per cluster of Ritz values (phases and
    # rotations inside a cluster are not unique), by the sine of the largest principal angle in the S inner
    # product, ||(I - U_o U_o^H S) U_g||_S over the cluster. Clusters are split where consecutive Ritz values
    # differ by more than gmin; Davis-Kahan bounds the angle by (perturbation) / (gap to the rest), about
    # 1e-12 / gmin here.
    gmin = 1e-4
    cuts = [0] + [i + 1 for i in range(len(lam) - 1) if lam[i + 1] - lam[i] > gmin] + [len(lam)]
    for a, b in zip(cuts[:-1], cuts[1:]):
        Uo, Ugc = U[:, a:b], Ug[:, a:b]
        D = Ugc - Uo @ (Uo.conj().T @ (ops.apply_S(Ugc)))
        sin = np.sqrt(max(np.linalg.eigvalsh(D.conj().T @ ops.apply_S(D)).max(), 0.0))
        assert sin < 1e-7, (a, b, sin)


@pytest.mark.parametrize("name", ["mid_paw", "mid_nc"])
def test_rayleigh_ritz_multi_tile(name):
    """150 bands: the Hermitian Grams take 3 x 3 tiles of 64 (6 on and above the diagonal, the last row and column
    ragged) and mirror the rest. Ritz values, residuals and S-orthonormality against the oracle, with and without
    an overlap."""
    pb = wl.make_problem(name, nb=150)
    ops = matfree.Operators.from_problem(pb)
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    Y = matfree.chebyshev_filter(ops, pb.X0, 2, 1.0, 3.0)
    lam, U, res = matfree.rayleigh_ritz(ops, Y)
    Yd = cf.to_device_block(Y, torch.complex128)
    ritz, rd = plan.rayleigh_ritz(Yd)
    ritz = ritz.cpu().numpy()
    assert np.all(np.abs(ritz - lam) <= 1e-10 * np.maximum(np.abs(lam), 1.0))
    assert np.allclose(rd.cpu().numpy(), res, rtol=1e-6, atol=1e-9)
    Ug = cf.to_host_block(Yd)
    assert np.allclose(Ug.conj().T @ ops.apply_S(Ug), np.eye(Ug.shape[1]), atol=1e-9)


def test_rayleigh_quotients_and_bound(case):
    pb, ops, plan = case
    Xd = cf.to_device_block(pb.X0, torch.complex128)
    rq = plan.rayleigh_quotients(Xd).cpu().numpy()
    assert np.allclose(rq, matfree.rayleigh_quotients(ops, pb.X0), rtol=1e-12, atol=1e-12)
    lp_ref = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lp = plan.upper_bound(torch.from_numpy(pb.v0), 10)
    assert abs(lp - lp_ref) <= 1e-10 * max(abs(lp_ref), 1.0)


@pytest.mark.parametrize("carry", [False, True], ids=["recomputed", "carried"])
def test_outer_loop_trajectory(case, carry):
    """The outer loop against the oracle's; with carry, the projections P^H X go from each filter and
    Rayleigh-Ritz call to the next instead of being recomputed (the oracle recomputes them every step)."""
    pb, ops, plan = case
    iters = min(pb.cfg.iters, 6)
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lam_o, _, res_o, hist_o = matfree.chebfsi(ops, pb.X0, pb.cfg.m, iters, lp)
    Xd = cf.to_device_block(pb.X0, torch.complex128)
    ritz, res, hist = chebfsi(plan, Xd, pb.cfg.m, iters, lp, carry=carry)
    for ho, hg in zip(hist_o, hist):
        assert abs(ho["lam_minus"] - hg["lam_minus"]) <= 1e-10 * max(abs(ho["lam_minus"]), 1.0)
        assert np.all(np.abs(hg["ritz"] - ho["ritz"]) <= 1e-10 * np.maximum(np.abs(ho["ritz"]), 1.0))


def test_carried_projections_match_recomputed(case):
    """cheb_rayleigh_ritz_carry returns P^H and (K + V) of its rotated block, with and without residuals;
    cheb_filter_carry started from them equals cheb_filter, in FP64 and in mixed plans."""
    pb, ops, plan = case
    nb, m = pb.cfg.nb, pb.cfg.m
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lm = float(np.max(matfree.rayleigh_quotients(ops, pb.X0)))
    c, r = 0.5 * (lp + lm), 0.5 * (lp - lm)
    PH = ops.P.conj().T if pb.nproj > 0 else None

    def local(Y):  # (K + V) Y
        return ops.kin[:, None] * Y + ops.vloc(Y)

    for with_res in (True, False):
        X = cf.to_device_block(pb.X0, torch.complex128)
        Xr = cf.to_device_block(pb.X0, torch.complex128)
        pz = plan.projections(nb)
        hz = torch.empty_like(X)
        ra, _ = plan.rayleigh_ritz(Xr, with_residuals=with_res)
        rb, _ = plan.rayleigh_ritz(X, with_residuals=with_res, p_out=pz, hx_out=hz)
        assert torch.equal(ra, rb) and torch.equal(X, Xr)
        if PH is not None:
            assert _rel(pz.cpu().numpy().T, PH @ cf.to_host_block(X)) < 1e-12
        assert _rel(cf.to_host_block(hz), local(cf.to_host_block(X))) < 1e-12
    # the filter from the returned quantities against the filter that computes them, and the oracle
    Xa = X.clone()
    plan.filter(Xa, m, c, r)
    Xb = X.clone()
    plan.filter(Xb, m, c, r, hx_in=hz)
    plan.filter(X, m, c, r, p_in=pz, hx_in=hz)
    for Y in (X, Xb):
        assert _rel(cf.to_host_block(Y), cf.to_host_block(Xa)) < 1e-11
    assert _rel(cf.to_host_block(X), matfree.chebyshev_filter(ops, cf.to_host_block(Xr), m, c, r)) < 1e-11
    # m = 0 leaves the block as it is
    Xa.copy_(X)
    plan.filter(Xa, 0, c, r, p_in=pz, hx_in=hz)
    assert torch.equal(Xa, X)
    # mixed plan: the quantities of the rotated complex64 block start the filter
    pm = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    Xm = cf.to_device_block(pb.X0, torch.complex64)
    pzm = pm.projections(nb)
    hzm = torch.empty_like(Xm)
    pm.rayleigh_ritz(Xm, p_out=pzm, hx_out=hzm)
    Y = cf.to_host_block(Xm)
    if PH is not None:
        assert _rel(pzm.cpu().numpy().T, PH @ Y) < 1e-6
    assert _rel(cf.to_host_block(hzm), local(Y)) < 1e-5
    ref = matfree.chebyshev_filter(ops, Y, m, c, r)
    Xn = Xm.clone()
    pm.filter(Xn, m, c, r)
    pm.filter(Xm, m, c, r, p_in=pzm, hx_in=hzm)
    assert _rel(cf.to_host_block(Xn), ref) < 1e-4
    assert _rel(cf.to_host_block(Xm), ref) < 1e-4
    # wrong buffers are refused by the binding; NULL ones are computed by the library
    with pytest.raises(ValueError):
        plan.filter(X, m, c, r, p_in=pz.to(torch.complex64))
    with pytest.raises(ValueError):
        plan.filter(X, m, c, r, hx_in=hz.to(torch.complex64))
    with pytest.raises(ValueError):
        plan.rayleigh_ritz(X, p_out=pz[: nb - 1])
    with pytest.raises(ValueError):
        plan.rayleigh_ritz(X, hx_out=hz[: nb - 1])
    Xc, Xd = X.clone(), X.clone()
    plan.filter(Xc, m, c, r)
    ws = plan.workspace(cf.CHEB_OP_FILTER, nb)
    st = plan.lib.cheb_filter_carry(plan.handle, Xd.data_ptr(), Xd.shape[1], nb, m, c, r, None, None, ws.data_ptr(),
                                    ws.numel(), cf._stream())
    assert st == 0 and torch.equal(Xc, Xd)


@pytest.mark.parametrize("split", [True, False], ids=["fp16x2-split", "fp32-mfma"])
def test_mixed_operators(case, split):
    """Mixed plans with the projector GEMMs on the FP16 hi/lo split MFMA (default) or the FP32 MFMA: both
    hold FP32-level accuracy, per band as well as over the block."""
    pb, ops, _ = case
    plan = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    plan.set_split_gemm(split)
    X = pb.X0
    Xd = cf.to_device_block(X, torch.complex64)
    for got, ref in ((plan.apply_H(Xd), ops.apply_H(X)), (plan.apply_Sinv(Xd), ops.apply_Sinv(X)),
                     (plan.apply_S(Xd), ops.apply_S(X))):
        got = cf.to_host_block(got)
        assert _rel(got, ref) < 2e-5
        colerr = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert colerr.max() < 4e-5
    # scaled bands: the per-band power-of-two scaling keeps huge and tiny columns as accurate
    scale = np.logspace(-6, 6, X.shape[1])
    Xs = X * scale[None, :]
    got = cf.to_host_block(plan.apply_Sinv(cf.to_device_block(Xs, torch.complex64)))
    ref = ops.apply_Sinv(Xs)
    colerr = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert colerr.max() < 4e-5


def test_rr_refinement_and_library_paths_agree(case):
    """The warm-started refinement and the library eigensolver give the same trajectory (and the oracle's)."""
    pb, ops, plan = case
    iters = 6
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    hist_o = matfree.chebfsi(ops, pb.X0, pb.cfg.m, iters, lp)[3]
    out = {}
    for on in (True, False):
        plan.set_rr_refine(on)
        r0, f0 = plan.rr_stats()
        Xd = cf.to_device_block(pb.X0, torch.complex128)
        out[on] = chebfsi(plan, Xd, pb.cfg.m, iters, lp)[2]
        r1, f1 = plan.rr_stats()
        print(f"refine={on}: refined {r1 - r0}, library {f1 - f0}")
        if not on:
            assert r1 == r0
    plan.set_rr_refine(True)
    for ho, h1, h0 in zip(hist_o, out[True], out[False]):
        tol = 1e-10 * np.maximum(np.abs(ho["ritz"]), 1.0)
        assert np.all(np.abs(h1["ritz"] - ho["ritz"]) <= tol)
        assert np.all(np.abs(h0["ritz"] - ho["ritz"]) <= tol)
