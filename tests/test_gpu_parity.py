"""GPU parity: every HIP path of libffth against the FP64 CPU oracle on the
same seeded inputs.  Tolerances: FP64 operator applications 1e-12 relative
L2 (rounding only); FP32 applications 5e-6; solves to residual 1e-10 versus
the oracle at 1e-12: strain fields 1e-6 relative L2 and effective stiffness
|dC_IJ| <= 1e-7 sqrt(C_II C_JJ)."""
import numpy as np
import pytest

from oracle import homogenization as H
from oracle import spectral, tensors
from paper_1712_05145_amd import ffth
from paper_1712_05145_amd import microstructure as M
from tests._gpu import full, rel_l2, require_gpu, to_dev, voigt6

pytestmark = pytest.mark.gpu

SIZES = [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256, 512, 1024]
# every size in every axis position, with small companions
SHAPES = sorted({s for n in SIZES for s in [(n, 6, 8), (8, n, 6), (6, 8, n)]})


def _uniform_solver(torch, shape, lam0=1.7, mu0=0.9, **kw):
    phase = np.zeros(shape, dtype=np.uint16)
    return ffth.Solver(phase, lam0, mu0, lame=[[2.0, 1.0]], **kw)


@pytest.mark.parametrize("shape", SHAPES)
def test_green_operator_fp64_all_sizes(shape):
    """eta = -Gamma0 * tau (x/y/z passes, Green operator, Nyquist and mean rules)."""
    torch = require_gpu()
    print("case green fp64", shape, flush=True)
    rng = np.random.default_rng(sum(shape))
    tau = rng.standard_normal((6,) + shape)
    ref = voigt6(spectral.green_apply(full(tau), 1.7, 0.9))
    s = _uniform_solver(torch, shape)
    got = s.green_apply(to_dev(torch, tau)).cpu().numpy()
    assert rel_l2(got, ref) < 1e-12


@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 48, 32), (64, 8, 96), (256, 6, 12)])
def test_green_operator_fp32(shape):
    torch = require_gpu()
    print("case green fp32", shape, flush=True)
    rng = np.random.default_rng(1)
    tau = rng.standard_normal((6,) + shape)
    ref = voigt6(spectral.green_apply(full(tau), 3.0, 1.2))
    s = _uniform_solver(torch, shape, lam0=3.0, mu0=1.2)
    got = s.green_apply(to_dev(torch, tau), precision="fp32").cpu().numpy()
    assert rel_l2(got, ref) < 5e-6


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 12, 16), (32, 24, 48)])
def test_displacement_recovery(shape):
    torch = require_gpu()
    print("case displacement", shape, flush=True)
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3,) + shape)
    eps = voigt6(spectral.sym_gradient(u))
    eps += 0.1 * rng.standard_normal(eps.shape)      # also an incompatible part
    ref = spectral.displacement_from_strain(full(eps))
    s = _uniform_solver(torch, shape)
    got = s.displacement(to_dev(torch, eps)).cpu().numpy()
    assert rel_l2(got, ref) < 1e-12


def _sphere(n, contrast=10.0):
    phase, lame = M.centred_sphere(n, young=(1.0, contrast))
    lam0, mu0 = M.midpoint_reference(lame)
    return phase, lame, lam0, mu0


@pytest.fixture(scope="module")
def sphere16_oracle():
    phase, lame, lam0, mu0 = _sphere(16)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    ceff, corr, infos = H.effective_stiffness(prob, "cg", tol=1e-12)
    return phase, lame, lam0, mu0, ceff, corr, infos


def _ceff_close(c_gpu, c_ref, tol=1e-7):
    d = np.sqrt(np.outer(np.diag(c_ref), np.diag(c_ref)))
    return np.abs(c_gpu - c_ref).max() / 1.0, np.all(np.abs(c_gpu - c_ref) <= tol * d)


@pytest.mark.parametrize("scheme,precision", [("basic", "fp64"), ("cg", "fp64"), ("cg", "mixed"),
                                              ("basic", "mixed")])
def test_order0_solve_parity_sphere16(sphere16_oracle, scheme, precision):
    """Config-1 geometry, six unit loads in one batched call."""
    torch = require_gpu()
    print("case order0", scheme, precision, flush=True)
    phase, lame, lam0, mu0, ceff, corr, _ = sphere16_oracle
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, scheme=scheme, precision=precision, tol=1e-10)
    eps, res = s.solve_order0(np.eye(6))
    eps = eps.cpu().numpy()
    cg = np.array([r["mean_stress"] for r in res]).T
    for J in range(6):
        assert res[J]["status"] == 0
        assert res[J]["residual"] < 1e-10
        assert rel_l2(eps[J], voigt6(corr[J])) < 1e-6, J
    _, ok = _ceff_close(cg, ceff)
    assert ok, np.abs(cg - ceff).max()


def test_order0_fp32_reports_floor(sphere16_oracle):
    """FP32-only runs stop at their rounding floor; the measured error is reported."""
    torch = require_gpu()
    phase, lame, lam0, mu0, ceff, corr, _ = sphere16_oracle
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=1, scheme="cg", precision="fp32", tol=1e-5)
    eps, res = s.solve_order0([1, 0, 0, 0, 0, 0])
    err = rel_l2(eps[0].cpu().numpy(), voigt6(corr[0]))
    print("fp32 cg field error", err, "iters", res[0]["iters"])
    assert res[0]["status"] == 0 and err < 1e-4


def test_basic_scheme_iteration_count_matches_oracle(sphere16_oracle):
    """The FP64 Basic Scheme follows the oracle's iterates: same count to the same tolerance."""
    torch = require_gpu()
    phase, lame, lam0, mu0, *_ = sphere16_oracle
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, _, info = H.solve_order0(prob, [1, 0, 0, 0, 0, 0], "basic", tol=1e-8)
    s = ffth.Solver(phase, lam0, mu0, lame=lame, scheme="basic", precision="fp64", tol=1e-8, check_every=1)
    _, res = s.solve_order0([1, 0, 0, 0, 0, 0])
    assert res[0]["iters"] == info["iters"]
    _, _, info_cg = H.solve_order0(prob, [1, 0, 0, 0, 0, 0], "cg", tol=1e-8)
    s2 = ffth.Solver(phase, lam0, mu0, lame=lame, scheme="cg", precision="fp64", tol=1e-8, check_every=1)
    _, res2 = s2.solve_order0([1, 0, 0, 0, 0, 0])
    assert abs(res2[0]["iters"] - info_cg["iters"]) <= 1


@pytest.mark.parametrize("shape,seed", [((12, 16, 8), 3), ((24, 12, 32), 4)])
def test_order0_noncubic_random_phases_ragged(shape, seed):
    """Non-cubic grids with a ragged last tile; three phases, generic stiffness rows."""
    torch = require_gpu()
    print("case noncubic", shape, flush=True)
    rng = np.random.default_rng(seed)
    phase = M.random_phases(shape, 3, seed)
    v21 = []
    for _ in range(3):
        a = rng.standard_normal((6, 6))
        c = a @ a.T + 6 * np.eye(6)
        v21.append([c[i, j] for i in range(6) for j in range(i, 6)])
    v21 = np.array(v21)
    lam0, mu0 = 3.0, 3.0
    prob = H.make_problem(phase, lam0, mu0, voigt21=v21)
    E = np.array([0.3, -1.0, 0.5, 0.2, 0.0, 1.0])
    eps_ref, mean_ref, _ = H.solve_order0(prob, E, "cg", tol=1e-12)
    s = ffth.Solver(phase, lam0, mu0, voigt21=v21, scheme="cg", precision="mixed", tol=1e-10)
    eps, res = s.solve_order0(E)
    assert rel_l2(eps[0].cpu().numpy(), voigt6(eps_ref)) < 1e-6
    assert np.allclose(res[0]["mean_stress"], mean_ref, rtol=1e-7, atol=1e-9 * np.abs(mean_ref).max())


def test_zero_rhs_reference_equals_material():
    torch = require_gpu()
    phase = np.zeros((8, 8, 8), dtype=np.uint16)
    for prec in ("fp64", "fp32", "mixed"):
        for scheme in ("basic", "cg", "bicgstab"):
            if prec == "mixed" and scheme == "bicgstab":
                continue
            s = ffth.Solver(phase, 1.3, 0.8, lame=[[1.3, 0.8]], scheme=scheme, precision=prec)
            eps, res = s.solve_order0([1.0, 0.5, 0, 0.2, 0, 0])
            assert res[0]["status"] == 0 and res[0]["iters"] == 0
            assert torch.count_nonzero(eps).item() == 0
            sig = tensors.stress_voigt_from_tensor(np.einsum(
                "ijkl,kl->ij", tensors.isotropic_stiffness(1.3, 0.8),
                tensors.tensor_from_engineering([1.0, 0.5, 0, 0.2, 0, 0])))
            assert np.allclose(res[0]["mean_stress"], sig, rtol=1e-12, atol=1e-14)


def test_batched_equals_single(sphere16_oracle):
    """A load solved alone and inside a batch of six gives the same field."""
    torch = require_gpu()
    phase, lame, lam0, mu0, *_ = sphere16_oracle
    s6 = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, tol=1e-9)
    eps6, _ = s6.solve_order0(np.eye(6))
    s1 = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=1, tol=1e-9)
    for J in (0, 4):
        e = np.zeros(6)
        e[J] = 1
        eps1, _ = s1.solve_order0(e)
        assert torch.equal(eps1[0], eps6[J])


def test_not_converged_reported():
    torch = require_gpu()
    phase, lame, lam0, mu0 = _sphere(16, contrast=100.0)
    s = ffth.Solver(phase, lam0, mu0, lame=lame, scheme="basic", precision="fp64", tol=1e-12, max_iter=5)
    eps, res = s.solve_order0([1, 0, 0, 0, 0, 0], check=False)
    assert res[0]["status"] == ffth.FFTH_ERR_NOT_CONVERGED and res[0]["iters"] == 5
    assert np.isfinite(eps.cpu().numpy()).all()


@pytest.fixture(scope="module")
def laminate_order1_case():
    n = 9 + 3   # even grid, even-thickness layers
    layers = [0, 0, 1, 1, 1, 1, 2, 2, 0, 0, 1, 1]
    phase = M.laminate((8, 6, n), layers, axis=2)
    lame = M.lame_from_young([1.0, 5.0, 2.5], [0.3, 0.25, 0.35])
    lam0, mu0 = M.midpoint_reference(lame)
    return phase, lame, lam0, mu0


def test_order1_rhs_and_solve_parity_sphere():
    """Order-1 right-hand side (X1, p2, g, theta) and solve against the oracle
    with identical order-0 correctors as input."""
    torch = require_gpu()
    print("case order1 sphere", flush=True)
    phase, lame, lam0, mu0 = _sphere(12)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.zeros((6, 3))
    grad[0, 0] = grad[1, 1] = 1.0                     # (grad E)_111 = (grad E)_222 = 1
    grad += 0.2 * np.random.default_rng(5).standard_normal((6, 3))
    p_ref, p2, theta, g, gmean = H.order1_rhs(prob, corr, grad)
    eps2_ref, info = H.solve_order1(prob, corr, grad, "cg", tol=1e-12)
    eps0 = to_dev(torch, np.stack([voigt6(c) for c in corr]))
    s = ffth.Solver(phase, lam0, mu0, lame=lame, order=1, nloads=1, tol=1e-10)
    pg, gm = s.order1_rhs(eps0, grad.reshape(18))
    assert rel_l2(pg.cpu().numpy(), voigt6(p_ref)) < 1e-12
    assert np.allclose(gm, gmean, rtol=1e-12, atol=1e-13)
    eps2, res = s.solve_order1(eps0, grad.reshape(1, 18))
    assert res[0]["status"] == 0
    assert rel_l2(eps2[0].cpu().numpy(), voigt6(eps2_ref)) < 1e-6
    # centrosymmetric cell: <C:eps2 + p2> vanishes; compare on the scale of p2
    assert np.allclose(res[0]["mean_stress"], info["mean_stress"], rtol=1e-7,
                       atol=1e-9 * np.abs(p2).max())
    assert np.allclose(res[0]["g_mean"], info["g_mean"], rtol=1e-12, atol=1e-13)


def test_order1_noncentrosymmetric_random_phases():
    """Random two-phase voxels (no symmetry): the order-1 mean stress is non-zero."""
    torch = require_gpu()
    shape = (12, 8, 16)
    phase = M.random_phases(shape, 2, 9)
    lame = M.lame_from_young([1.0, 8.0], [0.3, 0.3])
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.random.default_rng(10).standard_normal((6, 3))
    eps2_ref, info = H.solve_order1(prob, corr, grad, "cg", tol=1e-12)
    assert np.abs(info["mean_stress"]).max() > 1e-3
    eps0 = to_dev(torch, np.stack([voigt6(c) for c in corr]))
    s = ffth.Solver(phase, lam0, mu0, lame=lame, order=1, nloads=1, tol=1e-10)
    eps2, res = s.solve_order1(eps0, grad.reshape(1, 18))
    assert rel_l2(eps2[0].cpu().numpy(), voigt6(eps2_ref)) < 1e-6
    assert np.allclose(res[0]["mean_stress"], info["mean_stress"], rtol=1e-6,
                       atol=1e-8 * np.abs(info["mean_stress"]).max())


def test_order1_homogeneous_zero():
    torch = require_gpu()
    phase = np.zeros((8, 8, 8), dtype=np.uint16)
    s = ffth.Solver(phase, 2.0, 1.0, lame=[[1.0, 0.7]], order=1, nloads=1)
    eps0 = torch.zeros((6, 6, 8, 8, 8), dtype=torch.float64, device="cuda")
    grad = np.zeros(18)
    grad[0] = grad[4] = 1.0
    eps2, res = s.solve_order1(eps0, grad.reshape(1, 18))
    assert res[0]["iters"] == 0 and torch.count_nonzero(eps2).item() == 0


def test_order0_then_order1_chain(laminate_order1_case):
    """The order-1 solve consumes the GPU's own order-0 correctors (laminate)."""
    torch = require_gpu()
    phase, lame, lam0, mu0 = laminate_order1_case
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.random.default_rng(6).standard_normal((6, 3))
    eps2_ref, _ = H.solve_order1(prob, corr, grad, "cg", tol=1e-12)
    s0 = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, tol=1e-11)
    eps0, _ = s0.solve_order0(np.eye(6))
    s1 = ffth.Solver(phase, lam0, mu0, lame=lame, order=1, nloads=1, tol=1e-11)
    eps2, res = s1.solve_order1(eps0, grad.reshape(1, 18))
    assert rel_l2(eps2[0].cpu().numpy(), voigt6(eps2_ref)) < 1e-6


@pytest.mark.parametrize("scheme", ["cg", "basic"])
def test_mixed_laminate_reaches_tight_tolerance_backus(scheme):
    """Laminates make the FP32 inner solve exact in a few iterations, so later
    FP64 residuals are dominated by round-off outside the compatible subspace;
    the projected defect correction must still reach 1e-12 and the Backus C_eff."""
    torch = require_gpu()
    layers = [0, 0, 1, 1, 1, 1, 2, 2, 0, 0, 1, 1]
    phase = M.laminate((8, 6, 12), layers, axis=2)
    lame = M.lame_from_young([1.0, 5.0, 2.5], [0.3, 0.25, 0.35])
    lam0, mu0 = M.midpoint_reference(lame)
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, scheme=scheme, precision="mixed", tol=1e-12)
    _, res = s.solve_order0(np.eye(6))
    ceff = np.array([r["mean_stress"] for r in res]).T
    f = [np.mean(np.asarray(layers) == k) for k in range(3)]
    ref = H.laminate_backus(lame[:, 0], lame[:, 1], f)
    assert all(r["status"] == 0 for r in res), [r["outer_iters"] for r in res]
    assert np.abs(ceff - ref).max() < 1e-9 * np.abs(ref).max()



VARIANT_SHAPES = [(12, 24, 8), (64, 48, 32), (32, 128, 24), (24, 32, 128), (256, 12, 16), (16, 256, 8),
                  (16, 8, 256)]


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("shape", VARIANT_SHAPES)
def test_every_tile_variant_green_parity(variant, shape):
    """Each compiled tile shape of every pass gives the oracle's Gamma0 * tau."""
    torch = require_gpu()
    print("case green variant", variant, shape, flush=True)
    rng = np.random.default_rng(7 + sum(shape))
    tau = rng.standard_normal((6,) + shape)
    ref = voigt6(spectral.green_apply(full(tau), 1.7, 0.9))
    s = _uniform_solver(torch, shape, autotune=False)
    s.tile_variants = [variant] * 8
    assert s.tile_variants == [variant] * 8
    for precision, tol in (("fp64", 1e-12), ("fp32", 5e-6)):
        got = s.green_apply(to_dev(torch, tau), precision=precision).cpu().numpy()
        assert rel_l2(got, ref) < tol, (precision, rel_l2(got, ref))


def test_tile_variant_out_of_range_rejected():
    torch = require_gpu()
    s = _uniform_solver(torch, (8, 8, 8))
    with pytest.raises(ffth.FFTHError):
        s.tile_variants = [0, 0, 6, 0, 0, 0, 0, 0]
    assert s.tile_variants == [0] * 8


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("scheme", ["cg", "basic"])
def test_every_tile_variant_solve_parity(sphere16_oracle, variant, scheme):
    """Mixed solves with every pass on a non-default tile shape (all fused
    update and reduction modes) still match the oracle."""
    torch = require_gpu()
    print("case solve variant", variant, scheme, flush=True)
    phase, lame, lam0, mu0, ceff, corr, _ = sphere16_oracle
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, scheme=scheme, precision="mixed", tol=1e-10,
                    max_iter=5000)
    s.tile_variants = [variant] * 8
    eps, res = s.solve_order0(np.eye(6))
    eps = eps.cpu().numpy()
    assert all(r["status"] == 0 for r in res)
    for J in range(6):
        assert rel_l2(eps[J], voigt6(corr[J])) < 1e-6, J
    _, ok = _ceff_close(np.array([r["mean_stress"] for r in res]).T, ceff)
    assert ok


@pytest.mark.parametrize("scheme,precision", [("cg", "mixed"), ("basic", "mixed"), ("cg", "fp64"),
                                              ("bicgstab", "fp64"), ("cg3", "fp64"), ("cg3", "fp32"),
                                              ("cg", "mixed-binary16")])
def test_loads_per_launch_bit_identical(sphere16_oracle, scheme, precision):
    """Loads taken one and four at a time through every pass of an iteration
    (load-major order) give the results of one launch per pass bit for bit:
    each load's blocks and sums are the same in any launch.  The one-launch
    results match the oracle (the FP32-only solve at its own tolerance)."""
    torch = require_gpu()
    print("case launch loads", scheme, precision, flush=True)
    phase, lame, lam0, mu0, ceff, corr, _ = sphere16_oracle
    tol = 1e-5 if precision == "fp32" else 1e-10
    h16 = precision == "mixed-binary16"      # the binary16 spectrum forced on this small grid
    prec = "mixed" if h16 else precision
    out = {}
    for w in (0, 1, 4):
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, scheme=scheme, precision=prec, tol=tol,
                        max_iter=5000, autotune=False, spectrum16="force" if h16 else True)
        s.launch_loads = [w, w]
        assert s.launch_loads == [w, w]
        eps, res = s.solve_order0(np.eye(6))
        assert all(r["status"] == 0 for r in res), [r["status"] for r in res]
        out[w] = (eps.cpu().numpy(), np.array([r["mean_stress"] for r in res]), [r["iters"] for r in res])
        s.close()
    for w in (1, 4):
        assert np.array_equal(out[w][0], out[0][0]), w
        assert np.array_equal(out[w][1], out[0][1]), w
        assert out[w][2] == out[0][2], w
    bar = 1e-3 if precision == "fp32" else 1e-6
    for J in range(6):
        assert rel_l2(out[0][0][J], voigt6(corr[J])) < bar, J


def test_loads_per_launch_negative_rejected():
    torch = require_gpu()
    s = _uniform_solver(torch, (8, 8, 8))
    with pytest.raises(ffth.FFTHError):
        s.launch_loads = [-1, 0]
    assert s.launch_loads == [0, 0]


def test_autotuned_plan_matches_default_tiles():
    """The tuner's choice at 64^3 is a valid variant set and the solve agrees
    with the default tiles (same operator, reductions in another order)."""
    torch = require_gpu()
    print("case autotune 64", flush=True)
    phase, lame = M.random_spheres(64, 8, seed=5)
    lam0, mu0 = M.midpoint_reference(lame)
    out = {}
    for tune in (True, False):
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, precision="mixed", tol=1e-9, autotune=tune)
        v, w = s.tile_variants, s.launch_loads
        print("variants", tune, v, "loads per launch", w, flush=True)
        assert len(v) == 8 and all(0 <= x < ffth.TILE_VARIANTS for x in v)
        assert len(w) == 2 and all(0 <= x < 6 for x in w)
        if not tune:
            assert v == [0] * 8 and w == [0, 0]
        _, res = s.solve_order0(np.eye(6))
        assert all(r["status"] == 0 for r in res)
        out[tune] = np.array([r["mean_stress"] for r in res]).T
        s.close()
    d = np.sqrt(np.outer(np.diag(out[False]), np.diag(out[False])))
    assert np.all(np.abs(out[True] - out[False]) <= 1e-8 * d)


def test_mixed_three_term_inner_iterations_track_fp64_cg():
    """The FP32 inner solves (three-term CG restarted after each FP64 sweep)
    need about as many operator applications as plain FP64 CG."""
    torch = require_gpu()
    phase, lame = M.random_spheres(32, 6, seed=3)
    lam0, mu0 = M.midpoint_reference(lame)
    its = {}
    for precision in ("fp64", "mixed"):
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, precision=precision, tol=1e-8)
        _, res = s.solve_order0(np.eye(6))
        assert all(r["status"] == 0 and r["residual"] < 1e-8 for r in res)
        its[precision] = sum(r["iters"] for r in res)
    print("iterations", its)
    assert its["mixed"] <= 1.3 * its["fp64"] + 12


@pytest.mark.parametrize("tol,sweeps", [(1e-8, 4), (1e-10, 5), (1e-5, 3)])
def test_inner_targets_split_the_reduction(tol, sweeps):
    """The inner solves split the reduction the outer residual still needs over
    the fewest solves at the 1e-3 bound: ceil(log(0.8 tol) / log 1e-3) of them,
    so the FP64 applications per load are at most that count plus the right-hand
    side's (a solve that overshoots its target can save one)."""
    torch = require_gpu()
    print("case inner targets", tol, flush=True)
    phase, lame = M.random_spheres(32, 6, seed=3, young=(1.0, 20.0))
    lam0, mu0 = M.midpoint_reference(lame)
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, precision="mixed", tol=tol, inner_tol=1e-3)
    _, res = s.solve_order0(np.eye(6))
    print("fp64 applications", [r["fp64_applications"] for r in res], flush=True)
    assert all(r["status"] == 0 and r["residual"] < tol for r in res)
    assert all(r["fp64_applications"] <= sweeps for r in res)


def test_spectrum16_agrees_with_fp32_spectrum_and_is_gated():
    """Binary16 forward spectrum in the inner solve (128^3): same effective
    stiffness to the solve's accuracy and about the same iterations as the FP32
    spectrum when the stiffness contrast is within the limit; above it, and on
    grids below the size limit, the plan keeps FP32, so switching the option
    changes nothing (bit-identical results)."""
    torch = require_gpu()
    low = M.random_spheres(128, 6, seed=3, young=(1.0, 20.0))   # contrast 65
    high = M.overlapping_spheres(128, 0.25, 500.0, 7)           # contrast 1625
    small = M.random_spheres(64, 6, seed=3, young=(1.0, 20.0))
    assert ffth.ffth_stiffness_contrast(lame=low[1]) <= ffth.SPECTRUM16_MAX_CONTRAST
    assert ffth.ffth_stiffness_contrast(lame=high[1]) > ffth.SPECTRUM16_MAX_CONTRAST
    assert low[0].size >= ffth.SPECTRUM16_MIN_VOXELS > small[0].size
    for name, (phase, lame) in (("low", low), ("high", high), ("small", small)):
        print("case spectrum16", name, flush=True)
        lam0, mu0 = M.midpoint_reference(lame)
        out, its = {}, {}
        for h16 in (True, False):
            s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, precision="mixed", tol=1e-9, spectrum16=h16)
            _, res = s.solve_order0(np.eye(6))
            s.close()
            assert all(r["status"] == 0 and r["residual"] < 1e-9 for r in res)
            out[h16] = np.array([r["mean_stress"] for r in res]).T
            its[h16] = sum(r["iters"] for r in res)
        print("iterations", name, its, flush=True)
        if name == "low":
            d = np.sqrt(np.outer(np.diag(out[False]), np.diag(out[False])))
            assert np.all(np.abs(out[True] - out[False]) <= 1e-8 * d)
            assert its[True] <= 1.1 * its[False] + 8
            assert not np.array_equal(out[True], out[False])      # the binary16 path did run
        else:
            assert its[True] == its[False] and np.array_equal(out[True], out[False])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bicgstab_order0_parity_sphere16(sphere16_oracle, precision):
    """BiCGSTAB (the paper's solver) on the six unit loads in one batched call."""
    torch = require_gpu()
    print("case bicgstab order0", precision, flush=True)
    phase, lame, lam0, mu0, ceff, corr, _ = sphere16_oracle
    tol, ftol = (1e-10, 1e-6) if precision == "fp64" else (1e-5, 1e-4)
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, scheme="bicgstab", precision=precision, tol=tol)
    eps, res = s.solve_order0(np.eye(6))
    eps = eps.cpu().numpy()
    for J in range(6):
        assert res[J]["status"] == 0, res[J]
        assert rel_l2(eps[J], voigt6(corr[J])) < ftol, (J, rel_l2(eps[J], voigt6(corr[J])))
    if precision == "fp64":
        _, ok = _ceff_close(np.array([r["mean_stress"] for r in res]).T, ceff)
        assert ok


def test_bicgstab_iterations_and_residual_match_oracle():
    """Same iterates as the oracle's BiCGSTAB: iteration count and final residual."""
    torch = require_gpu()
    phase, lame, lam0, mu0 = _sphere(16, contrast=50.0)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    E = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    _, mean_ref, info = H.solve_order0(prob, E, "bicgstab", tol=1e-8)
    s = ffth.Solver(phase, lam0, mu0, lame=lame, scheme="bicgstab", precision="fp64", tol=1e-8, check_every=1)
    _, res = s.solve_order0(E)
    print("bicgstab iterations gpu", res[0]["iters"], "oracle", info["iters"])
    assert abs(res[0]["iters"] - info["iters"]) <= 1
    assert res[0]["residual"] < 1e-8
    assert res[0]["fp64_applications"] == 2 * res[0]["iters"] + 2


def test_bicgstab_generic_stiffness_and_order1():
    """Generic (anisotropic) phases on a non-cubic ragged grid, and the order-1
    problem, with BiCGSTAB in FP64."""
    torch = require_gpu()
    shape, seed = (12, 16, 8), 3
    rng = np.random.default_rng(seed)
    phase = M.random_phases(shape, 3, seed)
    v21 = []
    for _ in range(3):
        a = rng.standard_normal((6, 6))
        c = a @ a.T + 6 * np.eye(6)
        v21.append([c[i, j] for i in range(6) for j in range(i, 6)])
    v21 = np.array(v21)
    prob = H.make_problem(phase, 3.0, 3.0, voigt21=v21)
    E = np.array([0.3, -1.0, 0.5, 0.2, 0.0, 1.0])
    eps_ref, mean_ref, _ = H.solve_order0(prob, E, "cg", tol=1e-12)
    s = ffth.Solver(phase, 3.0, 3.0, voigt21=v21, scheme="bicgstab", precision="fp64", tol=1e-10)
    eps, res = s.solve_order0(E)
    assert rel_l2(eps[0].cpu().numpy(), voigt6(eps_ref)) < 1e-6
    assert np.allclose(res[0]["mean_stress"], mean_ref, rtol=1e-7, atol=1e-9 * np.abs(mean_ref).max())
    # order 1 from the oracle's correctors
    phase, lame, lam0, mu0 = _sphere(12)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.random.default_rng(8).standard_normal((6, 3))
    eps2_ref, _ = H.solve_order1(prob, corr, grad, "cg", tol=1e-12)
    eps0 = to_dev(torch, np.stack([voigt6(c) for c in corr]))
    s1 = ffth.Solver(phase, lam0, mu0, lame=lame, order=1, nloads=1, scheme="bicgstab", precision="fp64", tol=1e-10)
    eps2, res = s1.solve_order1(eps0, grad.reshape(1, 18))
    assert res[0]["status"] == 0
    assert rel_l2(eps2[0].cpu().numpy(), voigt6(eps2_ref)) < 1e-6


def test_bicgstab_mixed_rejected():
    torch = require_gpu()
    with pytest.raises(ffth.FFTHError):
        ffth.Solver(np.zeros((8, 8, 8), np.uint16), 1.0, 1.0, lame=[[1.0, 1.0]], scheme="bicgstab",
                    precision="mixed")
