"""The entry point that allocates nothing (cheb_apply_H_noalloc, static device scratch) against cheb_apply_H with a
caller workspace: the same kernels on the same inputs, so the results are identical, on two calls in a row, the
second with a smaller input; a block whose scratch would exceed the static array is refused before any launch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1406_4350_amd import chebfd as cf  # noqa: E402
from paper_1406_4350_amd import workload as wl  # noqa: E402


def _noalloc(plan, X, Y):
    nb, ldx = X.shape[0], X.stride(0)
    return plan.lib.cheb_apply_H_noalloc(plan.handle, ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(Y.data_ptr()),
                                         Y.stride(0), nb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("prec", [cf.CHEB_FP64, cf.CHEB_MIXED], ids=["fp64", "mixed"])
def test_noalloc_matches_workspace_entry(prec):
    dtype = torch.complex64 if prec == cf.CHEB_MIXED else torch.complex128
    big = wl.make_problem("paw48")
    small = wl.make_problem("mid_paw")
    print(f"[case] prec={prec}: paw48 64 bands, then paw48 17 bands, then mid_paw 40 bands", flush=True)
    pbig = cf.plan_from_problem(big, prec)
    psmall = cf.plan_from_problem(small, prec)
    for plan, pb, nb in ((pbig, big, 64), (pbig, big, 17), (psmall, small, small.cfg.nb)):
        X = cf.to_device_block(pb.X0[:, :nb], dtype)
        ref = plan.apply_H(X)
        Y = torch.full_like(X, float("nan"))
        assert _noalloc(plan, X, Y) == cf.CHEB_OK, plan.lib.cheb_last_error(plan.handle)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), float((Y - ref).abs().max())
    # more bands than the static scratch holds: refused, output untouched
    X = cf.to_device_block(big.X0, dtype)
    Y = torch.zeros_like(X)
    st = _noalloc(pbig, X, Y)
    assert st == cf.CHEB_ERR_WORKSPACE
    assert b"static scratch" in pbig.lib.cheb_last_error(pbig.handle)
    assert int(torch.count_nonzero(Y)) == 0
    pbig.close()
    psmall.close()
