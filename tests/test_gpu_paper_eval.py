"""The paper's own evaluation problem on the GPU path (Sec. 4): Hashin's coated
circular inclusion as a 2-D plane-stress problem on (1, n, n) grids (every
field invariant along x1, plane (x2, x3)), compared with the oracle; the
printed matrix modulus E3 = 453.685 makes the inclusion neutral."""
import json
import os

import numpy as np
import pytest

from oracle import homogenization as H
from oracle import spectral
from paper_1712_05145_amd import ffth
from paper_1712_05145_amd import microstructure as M
from tests._gpu import full, rel_l2, require_gpu, to_dev, voigt6

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# in-plane loads of the (x2, x3) plane: E22, E33, 2 E23 (engineering Voigt)
IN_PLANE = np.array([[0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0], [0, 0, 0, 1, 0, 0]], dtype=float)


@pytest.mark.parametrize("shape", [(1, 16, 24), (1, 64, 32), (1, 8, 1024), (1, 1024, 6)])
def test_green_operator_2d(shape):
    """A length-1 first axis: the z-pass applies the Green operator without a transform."""
    torch = require_gpu()
    print("case green 2d", shape, flush=True)
    rng = np.random.default_rng(sum(shape))
    tau = rng.standard_normal((6,) + shape)
    ref = voigt6(spectral.green_apply(full(tau), 1.3, 0.8))
    s = ffth.Solver(np.zeros(shape, np.uint16), 1.3, 0.8, lame=[[2.0, 1.0]])
    for precision, tol in (("fp64", 1e-12), ("fp32", 5e-6)):
        got = s.green_apply(to_dev(torch, tau), precision=precision).cpu().numpy()
        assert rel_l2(got, ref) < tol, (precision, rel_l2(got, ref))


@pytest.fixture(scope="module")
def hashin32_oracle():
    phase, lame = M.hashin_2d(32)
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    out = [H.solve_order0(prob, e, "cg", tol=1e-12) for e in IN_PLANE]
    return phase, lame, lam0, mu0, out


@pytest.mark.parametrize("scheme,precision,h16", [("cg", "fp64", False), ("basic", "fp64", False),
                                                  ("cg", "mixed", False), ("cg", "mixed", "force")])
def test_hashin2d_order0_parity(hashin32_oracle, scheme, precision, h16):
    """Sec. 4 structure at 32 x 32: strain fields and mean stresses of the three
    in-plane unit loads equal the oracle's (also with the binary16 forward
    spectrum forced on, as large grids run it)."""
    torch = require_gpu()
    print("case hashin2d order0", scheme, precision, h16, flush=True)
    phase, lame, lam0, mu0, ref = hashin32_oracle
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=3, scheme=scheme, precision=precision, tol=1e-10,
                    max_iter=20000, spectrum16=h16)
    eps, res = s.solve_order0(IN_PLANE)
    eps = eps.cpu().numpy()
    for J in range(3):
        assert res[J]["status"] == 0
        assert rel_l2(eps[J], voigt6(ref[J][0])) < 1e-6
        ms = np.asarray(ref[J][1])
        assert np.allclose(res[J]["mean_stress"], ms, rtol=1e-8, atol=1e-9 * np.abs(ms).max())
        # no x1 strain in a plane problem (round-off of the paired transforms only)
        assert np.abs(eps[J][0]).max() < 1e-14 * np.abs(eps[J]).max()


def test_hashin2d_order1_parity():
    """Order 1 on the 2-D structure: the paper's gradient load (grad E)_111 =
    (grad E)_222 = 1, mapped to the (x2, x3) plane, from the oracle's own
    correctors; field and mean stress equal the oracle's."""
    torch = require_gpu()
    print("case hashin2d order1", flush=True)
    phase, lame = M.hashin_2d(16)
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.zeros((6, 3))
    grad[1, 1] = grad[2, 2] = 1.0
    eps2_ref, info = H.solve_order1(prob, corr, grad, "cg", tol=1e-12)
    eps0 = to_dev(torch, np.stack([voigt6(c) for c in corr]))
    for scheme in ("cg", "basic"):
        s = ffth.Solver(phase, lam0, mu0, lame=lame, order=1, nloads=1, scheme=scheme, precision="fp64",
                        tol=1e-11, max_iter=50000)
        eps2, res = s.solve_order1(eps0, grad.reshape(1, 18))
        assert res[0]["status"] == 0
        assert rel_l2(eps2[0].cpu().numpy(), voigt6(eps2_ref)) < 1e-6
        assert np.allclose(res[0]["g_mean"], info["g_mean"], rtol=1e-10, atol=1e-12)


def test_hashin2d_neutral_inclusion_large_grids():
    """With the printed moduli the coated inclusion is neutral: the in-plane
    bulk modulus of the cell tends to the matrix's as the grid is refined."""
    torch = require_gpu()
    gold = json.load(open(os.path.join(GOLDEN, "hashin_2d.json")))
    errs = []
    for n in (128, 512, 1024):
        print("case hashin2d neutral", n, flush=True)
        phase, lame = M.hashin_2d(n, gold["r1"], gold["r2"],
                                  young=(gold["E1_core"], gold["E2_coating"], gold["E3_matrix"]), nu=gold["nu"])
        lam0, mu0 = M.midpoint_reference(lame)
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=1, precision="mixed", tol=1e-8)
        _, res = s.solve_order0([0, 1, 1, 0, 0, 0])
        s.close()
        ms = res[0]["mean_stress"]
        k_eff = (ms[1] + ms[2]) / 4.0
        k3 = lame[2, 0] + lame[2, 1]
        errs.append(abs(k_eff / k3 - 1))
    print("neutrality errors", errs)
    assert errs[0] < 0.02 * 32 / 128
    assert errs[2] < errs[0]


def test_coated_sphere_3d_neutral_inclusion():
    """3-D analogue of Sec. 4's structure: a coated sphere with the neutral
    matrix bulk modulus leaves the cell's bulk modulus at the matrix value."""
    torch = require_gpu()
    errs = []
    for n in (64, 128):
        print("case coated sphere", n, flush=True)
        young = np.array([100.0, 1000.0])
        lame = M.lame_from_young(young, [0.3, 0.3])
        k = lame[:, 0] + 2 * lame[:, 1] / 3
        f = (0.25 / 0.4) ** 3
        k3 = k[1] + f / (1 / (k[0] - k[1]) + 3 * (1 - f) / (3 * k[1] + 4 * lame[1, 1]))
        lame = np.vstack([lame, M.lame_from_young([3 * k3 * (1 - 2 * 0.3)], [0.3])])
        phase = M.coated_sphere(n)
        lam0, mu0 = M.midpoint_reference(lame)
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=1, precision="mixed", tol=1e-8)
        _, res = s.solve_order0([1, 1, 1, 0, 0, 0])
        s.close()
        k_eff = sum(res[0]["mean_stress"][:3]) / 9.0
        errs.append(abs(k_eff / k3 - 1))
    print("coated sphere neutrality errors", errs)
    assert max(errs) < 0.01
