"""Mixed precision (complex64 bands, FFTs and recurrence; FP16 hi/lo split projector GEMMs; FP64 subspace
matrices and dense eigensolver) against the FP64 oracle and the FP64 GPU path.

Rayleigh-Ritz of a mixed plan on a complex64 block: the subspace matrices are summed in FP64 from complex64
products, so their only error is the float32 rounding of H Y and S Y. With E_j the error of column j of H Y
(and F_j that of S Y), ||E_j|| <= C eps32 (||K y_j|| + ||V_loc y_j|| + ||P D P^H y_j||) and
||F_j|| <= C eps32 ||P Q P^H y_j|| (P itself is stored in complex64), the Ritz value of u_i = Y z_i moves by at
most ||u_i|| sum_j |z_ij| (||E_j|| + |lambda_i| ||F_j||) to first order. C = 64 covers the rounding steps of
the complex64 FFT pair (about 2 log2(n^3) of them at n <= 48) and of the split GEMMs.

The outer loop (Alg. 2) in mixed precision must reach the FP64 eigenpairs: over the lowest floor(0.8 nb)
bands, Ritz values within 1e-6 Ha of the converged FP64 path and residuals <= 1e-5 when the complex64 Ritz
vectors are re-evaluated with the FP64 operators.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import matfree  # noqa: E402
from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402
from paper_1406_4350_amd.driver import chebfsi  # noqa: E402

EPS32 = 2.0 ** -24
C_RND = 64.0


def _column_scales(ops, Y):
    """a_j = ||K y_j|| + ||V_loc y_j|| + ||P D P^H y_j||, b_j = ||P Q P^H y_j|| (0 without overlap)."""
    a = np.linalg.norm(ops.kin[:, None] * Y, axis=0) + np.linalg.norm(ops.vloc(Y), axis=0)
    b = np.zeros(Y.shape[1])
    if ops.P.shape[1]:
        p = ops.project(Y)
        a += np.linalg.norm(ops.P @ (ops.Dfull @ p), axis=0)
        if ops.Q is not None:
            b = np.linalg.norm(ops.P @ (ops.Q[:, None] * p), axis=0)
    return a, b


@pytest.mark.parametrize("name", ["nc16", "tiny_paw", "mid_paw", "mid_nc", "paw48"])
def test_mixed_rayleigh_ritz_parity(name):
    pb = wl.make_problem(name)
    print(f"[case] {name} npw={pb.npw} nb={pb.cfg.nb}", flush=True)
    ops = matfree.Operators.from_problem(pb)
    lp = matfree.lanczos_upper_bound(ops, pb.v0, 10)[0]
    lm = float(np.max(matfree.rayleigh_quotients(ops, pb.X0)))
    Y = matfree.chebyshev_filter(ops, pb.X0, pb.cfg.m, 0.5 * (lp + lm), 0.5 * (lp - lm))
    Y32 = Y.astype(np.complex64).astype(np.complex128)  # the block both sides see
    HY, SY = ops.apply_H(Y32), ops.apply_S(Y32)
    Hs, Ss = Y32.conj().T @ HY, Y32.conj().T @ SY
    import scipy.linalg
    lam, Z = scipy.linalg.eigh(0.5 * (Hs + Hs.conj().T), 0.5 * (Ss + Ss.conj().T))
    a, b = _column_scales(ops, Y32)
    unorm = np.linalg.norm(Y32 @ Z, axis=0)
    tau = C_RND * EPS32 * unorm * (np.abs(Z).T @ a + np.abs(lam) * (np.abs(Z).T @ b))
    plan = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    Yd = cf.to_device_block(Y32, torch.complex64)
    ritz, res = plan.rayleigh_ritz(Yd)
    ritz = ritz.cpu().numpy()
    err = np.abs(ritz - lam)
    print(f"[check] max |d lambda| {err.max():.3e}, max ratio to the rounding bound {np.max(err / tau):.3f}",
          flush=True)
    assert np.all(err <= tau)
    assert err.max() <= 1e-6  # the mixed-precision eigenvalue target, well above float32 rounding here
    # the rotated complex64 block is S-orthonormal to float32 rounding
    U = cf.to_host_block(Yd)
    G = U.conj().T @ ops.apply_S(U)
    assert np.abs(G - np.eye(U.shape[1])).max() < 1e-5


def _fp64_eval_residuals(p64, U32, lam):
    U = U32.to(torch.complex128)
    HU, SU = p64.apply_H(U), p64.apply_S(U)
    lt = torch.from_numpy(lam).to(U.device)
    return torch.linalg.vector_norm(HU - SU * lt[:, None], dim=1).cpu().numpy()


@pytest.mark.parametrize("name", ["mid_paw", "paw48", "paw96"])
def test_mixed_outer_loop_reaches_fp64_eigenpairs(name):
    pb = wl.make_problem(name)
    nb, m = pb.cfg.nb, pb.cfg.m
    k = int(0.8 * nb)
    print(f"[case] {name} npw={pb.npw} nb={nb} nproj={pb.nproj} m={m}, checked bands {k}", flush=True)
    p64 = cf.plan_from_problem(pb, cf.CHEB_FP64)
    lp = p64.upper_bound(torch.from_numpy(pb.v0), 10)
    # FP64 reference: iterate until the lowest k residuals are <= 1e-9
    X = cf.to_device_block(pb.X0, torch.complex128)
    lam64 = None
    for it in range(60):
        ritz, res, _ = chebfsi(p64, X, m, 1, lp) if it == 0 else _one_more(p64, X, m, lp, lam64)
        lam64, r64 = ritz.cpu().numpy(), res.cpu().numpy()
        if r64[:k].max() <= 1e-9:
            break
    print(f"[ref] FP64 converged after {it + 1} iterations, max residual {r64[:k].max():.2e}", flush=True)
    assert r64[:k].max() <= 1e-9
    pmx = cf.plan_from_problem(pb, cf.CHEB_MIXED)
    Xm = cf.to_device_block(pb.X0, torch.complex64)
    lamx = None
    for itm in range(60):
        ritz, res, _ = chebfsi(pmx, Xm, m, 1, lp) if itm == 0 else _one_more(pmx, Xm, m, lp, lamx)
        lamx = ritz.cpu().numpy()
        if itm >= it:  # at least as many iterations as the FP64 reference took
            rx = _fp64_eval_residuals(p64, Xm, lamx)
            if rx[:k].max() <= 1e-5 and np.abs(lamx[:k] - lam64[:k]).max() <= 1e-6:
                break
    dl = np.abs(lamx[:k] - lam64[:k])
    print(f"[mixed] {itm + 1} iterations: max |d lambda| {dl.max():.2e} Ha, max FP64-evaluated residual "
          f"{rx[:k].max():.2e}", flush=True)
    assert dl.max() <= 1e-6
    assert rx[:k].max() <= 1e-5


def _one_more(plan, X, m, lp, lam_prev):
    """One more outer iteration with lambda_- = the largest previous Ritz value."""
    lm = float(lam_prev.max())
    c, r = 0.5 * (lp + lm), 0.5 * (lp - lm)
    plan.filter(X, m, c, r)
    ritz, res = plan.rayleigh_ritz(X)
    return ritz, res, None
