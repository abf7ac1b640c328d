"""GPU parity of the exact kernel instantiations the 256^3 benchmark times,
against the FP64 oracle.

The benchmark's inner solve stores its forward spectrum in binary16 and runs
the passes on 256-point axes with the tile set the tuner picks there:
[x-forward FP32 2, x-forward FP64 0, y FP32 0, y FP64 1, z FP32 1, z FP64 1,
x-inverse FP32 0, x-inverse FP64 0] (variant 1 of the z-pass is a 2-column
tile, whose FP32 output after the Green operator takes the ordinary-store
branch).  Each grid below puts one 256-point axis in one position, so that
the binary16 z-pass (axis 0), the binary16 forward and FP32 inverse y-pass
(axis 1) and the fused three-term CG x-pass with its start pass (axis 2) of
the benchmark all run, with ragged last tiles in the other passes.  The
binary16 spectrum is forced on (the grids are below the size at which the
plan enables it by itself); the phases' stiffness contrast is within the
binary16 limit.

Bars: solves to residual 1e-10 versus the oracle's CG at 1e-12; strain
fields within 1e-6 relative L2; mean stresses within 1e-7 relative."""
import numpy as np
import pytest

from oracle import homogenization as H
from paper_1712_05145_amd import ffth
from paper_1712_05145_amd import microstructure as M
from tests._gpu import rel_l2, require_gpu, to_dev, voigt6

pytestmark = pytest.mark.gpu

BENCH_TILES = [2, 0, 0, 1, 1, 1, 0, 0]


def _grains(shape, seed, k=8):
    """k phases on random voxels with Lame pairs log-uniform in [1, 50] (the
    benchmark polycrystal's grain law)."""
    phase = M.random_phases(shape, k, seed)
    rng = np.random.default_rng(seed)
    lame = np.exp(rng.uniform(0.0, np.log(50.0), (k, 2)))
    lam0, mu0 = M.midpoint_reference(lame)
    assert ffth.ffth_stiffness_contrast(lame=lame) <= ffth.SPECTRUM16_MAX_CONTRAST
    return phase, lame, lam0, mu0


def _mean_close(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return np.all(np.abs(got - ref) <= 1e-7 * np.abs(ref).max())


@pytest.mark.parametrize("shape", [(256, 12, 16), (16, 256, 8), (16, 8, 256)])
def test_bench_binary16_instantiations_order0(shape):
    torch = require_gpu()
    print("case bench kernels order0", shape, flush=True)
    phase, lame, lam0, mu0 = _grains(shape, sum(shape))
    E = np.array([1.0, -0.4, 0.3, 0.5, -0.2, 0.8])
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    eps_ref, mean_ref, info = H.solve_order0(prob, E, "cg", tol=1e-12)
    assert info["converged"]
    out = {}
    for h16 in ("force", False):
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=1, precision="mixed", tol=1e-10, spectrum16=h16)
        s.tile_variants = BENCH_TILES
        eps, res = s.solve_order0(E)
        assert res[0]["status"] == 0 and res[0]["residual"] < 1e-10
        e = eps[0].cpu().numpy()
        assert rel_l2(e, voigt6(eps_ref)) < 1e-6, h16
        assert _mean_close(res[0]["mean_stress"], mean_ref), h16
        out[h16] = (e, res[0])
        s.close()
    # the binary16 kernels did run: the iterates differ from the FP32 spectrum's
    assert not np.array_equal(out["force"][0], out[False][0])


def test_bench_binary16_instantiations_order1():
    """Order-1 mixed solve with the benchmark's 256-point x-passes (fused CG
    pass and start pass in binary16), from the oracle's own correctors."""
    torch = require_gpu()
    shape = (8, 6, 256)
    print("case bench kernels order1", shape, flush=True)
    phase, lame, lam0, mu0 = _grains(shape, 31)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.zeros((6, 3))
    grad[0, 0] = grad[1, 1] = 1.0
    grad += 0.3 * np.random.default_rng(4).standard_normal((6, 3))
    eps2_ref, info = H.solve_order1(prob, corr, grad, "cg", tol=1e-12)
    eps0 = to_dev(torch, np.stack([voigt6(c) for c in corr]))
    s = ffth.Solver(phase, lam0, mu0, lame=lame, order=1, nloads=1, precision="mixed", tol=1e-10,
                    spectrum16="force")
    s.tile_variants = BENCH_TILES
    eps2, res = s.solve_order1(eps0, grad.reshape(1, 18))
    assert res[0]["status"] == 0
    assert rel_l2(eps2[0].cpu().numpy(), voigt6(eps2_ref)) < 1e-6
    assert _mean_close(res[0]["mean_stress"], info["mean_stress"])
    assert np.allclose(res[0]["g_mean"], info["g_mean"], rtol=1e-10, atol=1e-12 * np.abs(info["g_mean"]).max())
