"""The allocation-free Green operator application (ffth_green_apply_noalloc)
against the plan-based entry point (ffth_green_apply) through the C-ABI: two
calls in a row on one stream, the second on a smaller grid, in FP64 and FP32.
The two entry points run the same kernels in the same tile shapes, so the
results agree to rounding (bar: FP64 1e-12, FP32 5e-6 relative L2, as for
the Green operator parity against the oracle)."""
import ctypes

import numpy as np
import pytest

from paper_1712_05145_amd import ffth
from tests._gpu import rel_l2, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _plan_green(torch, shape, lam0, mu0, tau, precision):
    s = ffth.Solver(np.zeros(shape, np.uint16), lam0, mu0, lame=[[2.0, 1.0]])
    out = s.green_apply(tau, precision=precision)
    s.close()
    return out


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 5e-6)])
def test_noalloc_green_equals_plan_entry_point_twice(precision, tol):
    torch = require_gpu()
    stream = torch.cuda.current_stream()
    for k, (shape, lam0, mu0) in enumerate([((32, 48, 64), 1.7, 0.9), ((16, 12, 8), 3.0, 1.2)]):
        print("case noalloc", precision, shape, flush=True)
        rng = np.random.default_rng(k + 11)
        tau = to_dev(torch, rng.standard_normal((6,) + shape))
        ref = _plan_green(torch, shape, lam0, mu0, tau, precision)
        eta = torch.full_like(tau, float("nan"))
        ffth.ffth_green_apply_noalloc(shape, lam0, mu0, ffth._dptr(tau), ffth._dptr(eta),
                                      ffth.PRECISIONS[precision], ctypes.c_void_p(stream.cuda_stream))
        torch.cuda.synchronize()
        assert torch.isfinite(eta).all()
        assert rel_l2(eta.cpu().numpy(), ref.cpu().numpy()) <= tol


def test_noalloc_green_rejects_oversize_grid():
    torch = require_gpu()
    shape = (64, 64, 128)
    tau = torch.zeros((6,) + shape, dtype=torch.float64, device="cuda")
    with pytest.raises(ffth.FFTHError) as e:
        ffth.ffth_green_apply_noalloc(shape, 1.0, 1.0, ffth._dptr(tau), ffth._dptr(tau))
    assert e.value.status == ffth.FFTH_ERR_INVALID and "exceeds" in str(e.value)
