"""Per-section event timers (cheb_profile_enable / cheb_profile_read).

The sections are disjoint intervals on the plan's stream, so over outer iterations of filter + Rayleigh-Ritz
(Alg. 2) their times add up to no more than the wall time of those iterations; every section of the path is
hit, and a section timed in two intervals (the rotation around the residual back-projection) still counts one
launch per call.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402


@pytest.mark.parametrize("prec", [cf.CHEB_FP64, cf.CHEB_MIXED], ids=["fp64", "mixed"])
def test_sections_disjoint_and_counted(prec):
    pb = wl.make_problem("mid_paw")
    print(f"[case] {pb.cfg.name} prec={prec} npw={pb.npw} nb={pb.cfg.nb}", flush=True)
    plan = cf.plan_from_problem(pb, prec)
    X = cf.to_device_block(pb.X0, torch.complex64 if prec == cf.CHEB_MIXED else torch.complex128)
    lam_plus = plan.upper_bound(torch.from_numpy(pb.v0), 10)
    lam_minus = float(plan.rayleigh_quotients(X).max().item())
    m, steps = pb.cfg.m, 3

    def step(lam_minus):
        c, r = 0.5 * (lam_plus + lam_minus), 0.5 * (lam_plus - lam_minus)
        plan.filter(X, m, c, r)
        ritz, _ = plan.rayleigh_ritz(X)
        return float(ritz.max().item())

    lam_minus = step(lam_minus)
    torch.cuda.synchronize()
    plan.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        lam_minus = step(lam_minus)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    prof = plan.profile_read()
    plan.profile_enable(False)

    total = sum(v["ms"] for v in prof.values())
    assert 0.0 < total <= wall_ms * 1.01 + 0.05, (total, wall_ms, prof)
    for name in ("fft_col_inverse", "fft_plane", "fft_col_forward", "project", "backproject", "rr_gram", "rr_eig",
                 "rr_rotate"):
        assert prof[name]["launches"] >= steps and prof[name]["ms"] > 0.0, (name, prof[name])
    assert prof["rr_gram"]["launches"] == steps
    assert prof["rr_rotate"]["launches"] == steps
    assert np.isfinite(lam_minus)
