"""Edge cases and error paths of the HIP path through the C ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import dense, matfree  # noqa: E402
from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def tiny():
    pb = wl.make_problem("tiny_paw")
    return pb, matfree.Operators.from_problem(pb), cf.plan_from_problem(pb, cf.CHEB_FP64)


def test_single_band_and_empty_block(tiny):
    pb, ops, plan = tiny
    X = pb.X0[:, :1]
    Xd = cf.to_device_block(X, torch.complex128)
    assert _rel(cf.to_host_block(plan.apply_H(Xd)), ops.apply_H(X)) < 1e-12
    empty = torch.empty((0, pb.npw), dtype=torch.complex128, device="cuda")
    plan.apply_H(empty)
    plan.filter(empty, 3, 1.0, 2.0)


def test_padded_leading_dimension(tiny):
    """ldx > npw: bands are rows of a wider buffer; padding must stay untouched."""
    pb, ops, plan = tiny
    pad = 37
    buf = torch.full((pb.cfg.nb, pb.npw + pad), 7.0 + 3.0j, dtype=torch.complex128, device="cuda")
    buf[:, :pb.npw] = cf.to_device_block(pb.X0, torch.complex128)
    Xv = buf[:, :pb.npw]
    out = torch.full_like(buf, -1.0)
    plan.apply_H(Xv, out[:, :pb.npw])
    assert _rel(cf.to_host_block(out[:, :pb.npw]), ops.apply_H(pb.X0)) < 1e-12
    assert torch.all(out[:, pb.npw:] == -1.0)
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    plan.filter(Xv, 4, 0.5 * (lp + 1.0), 0.5 * (lp - 1.0))
    ref = matfree.chebyshev_filter(ops, pb.X0, 4, 0.5 * (lp + 1.0), 0.5 * (lp - 1.0))
    assert _rel(cf.to_host_block(Xv), ref) < 1e-11
    assert torch.all(buf[:, pb.npw:] == 7.0 + 3.0j)
    # the carried-projection entry points on the same padded rows: Rayleigh-Ritz returns P^H of its rotated block
    # and the filter starts from it
    Y = cf.to_host_block(Xv)
    pz = plan.projections(pb.cfg.nb)
    plan.rayleigh_ritz(Xv, p_out=pz)
    Yr = cf.to_host_block(Xv)
    assert _rel(pz.cpu().numpy().T, ops.P.conj().T @ Yr) < 1e-12
    lam, _, _ = matfree.rayleigh_ritz(ops, Y)
    c, r = 0.5 * (lp + lam.max()), 0.5 * (lp - lam.max())
    plan.filter(Xv, 3, c, r, p_in=pz)
    assert _rel(cf.to_host_block(Xv), matfree.chebyshev_filter(ops, Yr, 3, c, r)) < 1e-11
    assert torch.all(buf[:, pb.npw:] == 7.0 + 3.0j)


def test_free_electron_spectrum_on_gpu():
    """No projectors, V = 0: the filter + Rayleigh-Ritz loop converges to the kinetic shells."""
    fe = wl.free_electron("nc16")
    plan = cf.Plan(fe.gidx, fe.kin, fe.cfg.n, fe.proj_off, False)
    plan.set_potential(torch.zeros((16, 16, 16), dtype=torch.float64))
    plan.set_projectors(torch.zeros((0, fe.npw), dtype=torch.complex128), None)
    plan.set_D(torch.zeros(0, dtype=torch.float64))
    X = cf.to_device_block(fe.X0, torch.complex128)
    from paper_1406_4350_amd.driver import chebfsi
    ritz, res, _ = chebfsi(plan, X, 8, 30, 3.2)
    lam = np.sort(fe.kin)[:16]
    r = ritz.cpu().numpy()
    assert np.all(np.abs(r[:7] - lam[:7]) < 1e-10)


# (128, 40): the largest sphere whose x-lines fit the halved FP64 plane of the 128 box (81 x-lines)
@pytest.mark.parametrize("n,radius", [(8, 3), (12, 2), (24, 11), (48, 6), (64, 8), (96, 10), (128, 12), (128, 40)])
def test_other_box_sizes(n, radius):
    cfg = wl.SMALL["tiny_paw"].replace(name=f"box{n}", n=n, radius=radius, nb=9, seed_index=200 + n)
    pb = wl.make_problem(cfg)
    ops = matfree.Operators.from_problem(pb)
    for prec, tol in ((cf.CHEB_FP64, 1e-12), (cf.CHEB_MIXED, 2e-5)):
        plan = cf.plan_from_problem(pb, prec)
        dt = torch.complex64 if prec == cf.CHEB_MIXED else torch.complex128
        Xd = cf.to_device_block(pb.X0, dt)
        assert _rel(cf.to_host_block(plan.apply_H(Xd)), ops.apply_H(pb.X0)) < tol


def test_box128_without_single_column_edge_lines():
    """A sphere of integer radius has one column (gy = 0) on each outermost x-line, which the FP64 plane pass at
    128^3 sets and sums directly; without the points (+-R, 0, 0) the basis has no such lines and every x-line
    takes the transforms. Both forms against the oracle, FP64 and mixed."""
    import dataclasses

    cfg = wl.SMALL["tiny_paw"].replace(name="box128e", n=128, radius=12, nb=9, seed_index=329)
    full = wl.make_problem(cfg)
    g = full.gidx
    keep = ~((np.abs(g[:, 0]) == 12) & (g[:, 1] == 0) & (g[:, 2] == 0))
    assert keep.sum() == full.npw - 2
    cut = dataclasses.replace(full, gidx=np.ascontiguousarray(g[keep]), kin=full.kin[keep],
                              P=np.asfortranarray(full.P[keep]), X0=np.asfortranarray(full.X0[keep]),
                              v0=full.v0[keep])
    for pb in (full, cut):
        ops = matfree.Operators.from_problem(pb)
        ref = ops.apply_H(pb.X0)
        for prec, tol in ((cf.CHEB_FP64, 1e-12), (cf.CHEB_MIXED, 2e-5)):
            plan = cf.plan_from_problem(pb, prec)
            dt = torch.complex64 if prec == cf.CHEB_MIXED else torch.complex128
            assert _rel(cf.to_host_block(plan.apply_H(cf.to_device_block(pb.X0, dt))), ref) < tol


@pytest.mark.parametrize("qscale", [1.0, 0.01], ids=["q", "q_small"])
def test_filter_with_small_overlap_coefficients(qscale):
    """With an overlap the filter's projector-space step uses w = C^-1 (Q^-1 D p - p_loc) and P^H S^-1 H psi =
    Q^-1 (D p - w) (C = Q^-1 + P^H P); its rounding grows with 1 / min |Q_i|. Overlap coefficients 100x smaller
    than the workloads' (1 / Q up to 1000) keep the FP64 filter within the parity bound against the oracle."""
    import dataclasses

    pb = wl.make_problem("tiny_paw")
    pb = dataclasses.replace(pb, Q=pb.Q * qscale)
    ops = matfree.Operators.from_problem(pb)
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lm = float(np.max(matfree.rayleigh_quotients(ops, pb.X0)))
    c, r = 0.5 * (lp + lm), 0.5 * (lp - lm)
    Xd = cf.to_device_block(pb.X0, torch.complex128)
    plan.filter(Xd, pb.cfg.m, c, r)
    ref = matfree.chebyshev_filter(ops, pb.X0, pb.cfg.m, c, r)
    assert _rel(cf.to_host_block(Xd), ref) < 1e-11


def test_error_paths(tiny):
    pb, ops, plan = tiny
    Xd = cf.to_device_block(pb.X0, torch.complex128)
    with pytest.raises(cf.ChebError) as e:  # aliasing input/output
        plan.apply_H(Xd, Xd)
    assert e.value.status == cf.CHEB_ERR_ARG
    with pytest.raises(cf.ChebError) as e:  # r <= 0
        plan.filter(Xd.clone(), 3, 1.0, 0.0)
    assert e.value.status == cf.CHEB_ERR_ARG
    Y = Xd.clone()
    Y[3] = Y[1]  # rank-deficient block
    with pytest.raises(cf.ChebError) as e:
        plan.rayleigh_ritz(Y)
    assert e.value.status in (cf.CHEB_ERR_NOT_PD, cf.CHEB_ERR_EIG)
    Z = Xd.clone()
    Z[2].zero_()  # zero column: caught before the eigensolver
    with pytest.raises(cf.ChebError) as e:
        plan.rayleigh_ritz(Z)
    assert e.value.status == cf.CHEB_ERR_NOT_PD
    ws = plan.workspace(cf.CHEB_OP_H, pb.cfg.nb)
    Yd = torch.empty_like(Xd)
    st = plan.lib.cheb_apply_H(plan.handle, Xd.data_ptr(), pb.npw, Yd.data_ptr(), pb.npw, pb.cfg.nb, ws.data_ptr(),
                               16, torch.cuda.current_stream().cuda_stream)
    assert st == cf.CHEB_ERR_WORKSPACE


def test_nonfinite_potential():
    pb = wl.make_problem("tiny_paw")
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    V = torch.from_numpy(pb.V.copy())
    V[1, 2, 3] = float("nan")
    plan.set_potential(V)
    with pytest.raises(cf.ChebError) as e:
        plan.rayleigh_ritz(cf.to_device_block(pb.X0, torch.complex128))
    assert e.value.status in (cf.CHEB_ERR_NONFINITE, cf.CHEB_ERR_NOT_PD)


def test_state_errors():
    pb = wl.make_problem("tiny_paw")
    plan = cf.Plan(pb.gidx, pb.kin, pb.cfg.n, pb.proj_off, True)
    with pytest.raises(cf.ChebError) as e:
        plan.apply_H(cf.to_device_block(pb.X0, torch.complex128))
    assert e.value.status == cf.CHEB_ERR_STATE


def test_filter_matches_spectral_closed_form():
    """GPU filter against T_m(S^-1 H) X = V T_m(Lambda) V^H S X from the dense pencil (Sec. 4.2)."""
    pb = wl.make_problem("tiny_paw")
    H = dense.hamiltonian(pb.gidx, pb.kin, pb.V, pb.P, pb.D)
    S = dense.overlap(pb.npw, pb.P, pb.Q)
    lam = dense.eig_pencil(H, S)[0]
    c, r = 0.5 * (lam[-1] + lam[20]), 0.5 * (lam[-1] - lam[20])
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    for m in (1, 4, 7):
        Xd = cf.to_device_block(pb.X0, torch.complex128)
        plan.filter(Xd, m, c, r)
        ref = dense.filter_spectral(H, S, pb.X0, m, c, r)
        assert _rel(cf.to_host_block(Xd), ref) < 1e-11
