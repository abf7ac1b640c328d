"""GPU parity at the benchmark sizes (256^3 Voronoi, 128^3 random spheres,
512^3 fibres) in the launch configuration bench.py times.  The oracle cannot
run full solves there, so these tests compare sampled outputs that the
oracle computes one by one (single Fourier modes, analytic correctors) and
properties that hold at any size (symmetry and bounds of C_eff, BS = CG,
mixed = FP64, residuals)."""
import numpy as np
import pytest

from oracle import homogenization as H
from oracle import spectral, tensors
from paper_1712_05145_amd import ffth
from paper_1712_05145_amd import microstructure as M
from tests._gpu import require_gpu

pytestmark = pytest.mark.gpu

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def _modes_field(n, modes, torch):
    """tau = sum_m Re(T_m exp(i 2 pi k_m . y)) on the grid (y at voxel centres)."""
    y = torch.tensor(-0.5 + (np.arange(n) + 0.5) / n, dtype=torch.float64, device="cuda")
    g0, g1, g2 = torch.meshgrid(y, y, y, indexing="ij")
    tau = torch.zeros((6, n, n, n), dtype=torch.float64, device="cuda")
    for k, amp in modes:
        ph = 2 * np.pi * (k[0] * g0 + k[1] * g1 + k[2] * g2)
        c, s = torch.cos(ph), torch.sin(ph)
        for a in range(6):
            tau[a] += amp[a].real * c - amp[a].imag * s
    return tau


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-6)])
def test_green_operator_256_single_modes(precision, tol):
    """eta = -Gamma0 * tau for a sum of Fourier modes (incl. a Nyquist-index mode,
    which must vanish) at 256^3, sampled against the oracle's Gamma0_hat."""
    torch = require_gpu()
    n = 256
    lam0, mu0 = 12.0, 7.5
    rng = np.random.default_rng(0)
    modes = []
    for k in [(1, 0, 0), (3, -5, 7), (0, 0, 127), (-40, 17, 2), (128, 3, 1)]:
        a = rng.standard_normal(6) + 1j * rng.standard_normal(6)
        modes.append((k, a))
    tau = _modes_field(n, modes, torch)
    s = ffth.Solver(np.zeros((n, n, n), np.uint16), lam0, mu0, lame=[[1.0, 1.0]])
    eta = s.green_apply(tau, precision=precision)
    # expected amplitudes: -Gamma0_hat(xi) : T for each retained mode; Nyquist (k0 = 128) -> 0
    expect_modes = []
    for k, a in modes:
        if abs(k[0]) == n // 2:
            continue
        g = spectral.gamma0_hat(2 * np.pi * np.array(k, float).reshape(3, 1), lam0, mu0)[..., 0]
        t = np.zeros((3, 3), complex)
        for c, (i, j) in enumerate(VOIGT):
            t[i, j] = t[j, i] = a[c]
        e = -np.einsum("ijkl,kl->ij", g, t)
        expect_modes.append((k, np.array([e[i, j] for (i, j) in VOIGT])))
    ref = _modes_field(n, expect_modes, torch)
    idx = torch.randint(0, n, (3, 4096), device="cuda")
    got_s = eta[:, idx[0], idx[1], idx[2]]
    ref_s = ref[:, idx[0], idx[1], idx[2]]
    err = torch.linalg.vector_norm(got_s - ref_s) / torch.linalg.vector_norm(ref_s)
    assert err.item() < tol, err.item()


def _ceff(res):
    return np.array([r["mean_stress"] for r in res]).T


def _check_ceff_properties(prob_lame, phase, ceff, tol):
    lam, mu = prob_lame[:, 0], prob_lame[:, 1]
    s = np.abs(ceff).max()
    assert np.abs(ceff - ceff.T).max() < tol * s
    # Voigt / Reuss bounds from phase fractions
    counts = np.bincount(phase.ravel(), minlength=len(lam)).astype(float)
    f = counts / counts.sum()
    cv = np.zeros((6, 6))
    sr = np.zeros((6, 6))
    for p in range(len(lam)):
        if f[p] == 0:
            continue
        c = tensors.voigt66_from_stiffness(tensors.isotropic_stiffness(lam[p], mu[p]))
        cv += f[p] * c
        sr += f[p] * np.linalg.inv(c)
    assert np.linalg.eigvalsh(cv - 0.5 * (ceff + ceff.T)).min() > -tol * s
    assert np.linalg.eigvalsh(0.5 * (ceff + ceff.T) - np.linalg.inv(sr)).min() > -tol * s


def test_voronoi256_bench_workload_mixed_vs_fp64():
    """The benchmark workload: six order-0 loads at 256^3, mixed vs plain FP64."""
    torch = require_gpu()
    print("case voronoi256", flush=True)
    phase, lame = M.voronoi_polycrystal(256, 200, 3)
    lam0, mu0 = M.midpoint_reference(lame)
    sm = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, precision="mixed", tol=1e-8)
    em, rm = sm.solve_order0(np.eye(6))
    cm = _ceff(rm)
    del sm
    sd = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, precision="fp64", tol=1e-8)
    ed, rd = sd.solve_order0(np.eye(6))
    cd = _ceff(rd)
    assert all(r["status"] == 0 and r["residual"] < 1e-8 for r in rm + rd)
    d = np.sqrt(np.outer(np.diag(cd), np.diag(cd)))
    assert np.all(np.abs(cm - cd) <= 1e-7 * d), np.abs(cm - cd).max()
    # field agreement (both at residual 1e-8; contrast <= 50)
    rel = (torch.linalg.vector_norm(em - ed) / torch.linalg.vector_norm(ed)).item()
    assert rel < 1e-6, rel
    _check_ceff_properties(lame, phase, cm, 1e-7)


def test_random_spheres128_bs_equals_cg_mixed():
    """128^3, 20 random spheres, contrast 100: BS and CG (mixed) reach the same C_eff."""
    torch = require_gpu()
    print("case spheres128", flush=True)
    phase, lame = M.random_spheres(128, 20, seed=2)
    lam0, mu0 = M.midpoint_reference(lame)
    out = {}
    for scheme in ("cg", "basic"):
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, scheme=scheme, precision="mixed", tol=1e-8,
                        max_iter=50000)
        _, res = s.solve_order0(np.eye(6))
        assert all(r["status"] == 0 for r in res), [r["status"] for r in res]
        out[scheme] = (_ceff(res), sum(r["iters"] for r in res))
    c1, c2 = out["cg"][0], out["basic"][0]
    d = np.sqrt(np.outer(np.diag(c1), np.diag(c1)))
    assert np.all(np.abs(c1 - c2) <= 2e-7 * d), np.abs(c1 - c2).max()
    assert out["cg"][1] < out["basic"][1] / 3          # CG << BS at contrast 100
    _check_ceff_properties(lame, phase, c1, 1e-7)


def _trig_correctors(n, amp):
    """eps^J_mm = 2 pi a_Jm cos(2 pi y_m): symmetric gradients of u_m = a_Jm sin(2 pi y_m)."""
    y = -0.5 + (np.arange(n) + 0.5) / n
    g = np.meshgrid(y, y, y, indexing="ij")
    out = np.zeros((6, 3, 3, n, n, n))
    for J in range(6):
        for m in range(3):
            out[J, m, m] = 2 * np.pi * amp[J, m] * np.cos(2 * np.pi * g[m])
    return out


def test_order1_rhs_256_against_coarse_exact_oracle():
    """Order-1 right-hand side P = p_2 + theta_2 at 256^3.  With a homogeneous
    material and correctors that are symmetric gradients of degree-1
    trigonometric displacements, P is a degree-1 trigonometric polynomial: the
    oracle computes it exactly on an 8^3 grid, and its interpolant at sampled
    256^3 voxel centres is the expected value."""
    torch = require_gpu()
    rng = np.random.default_rng(3)
    amp = rng.standard_normal((6, 3))
    grad = rng.standard_normal((6, 3))
    lame = np.array([[2.0, 1.5]])
    # oracle on 8^3
    nc = 8
    prob = H.make_problem(np.zeros((nc, nc, nc), np.uint16), 3.0, 2.0, lame=lame)
    corr = list(_trig_correctors(nc, amp))
    p_ref, _, _, _, gmean_ref = H.order1_rhs(prob, corr, grad)
    coef = np.fft.fftn(tensors.voigt6_from_field(p_ref), axes=(1, 2, 3)) / nc ** 3
    ks = [k for k in np.ndindex(nc, nc, nc) if np.abs(coef[(slice(None),) + k]).max() > 1e-12]
    # GPU at 256^3
    n = 256
    y = torch.tensor(-0.5 + (np.arange(n) + 0.5) / n, dtype=torch.float64, device="cuda")
    g = torch.meshgrid(y, y, y, indexing="ij")
    eps0 = torch.zeros((6, 6, n, n, n), dtype=torch.float64, device="cuda")
    for J in range(6):
        for m in range(3):
            eps0[J, m] = 2 * np.pi * amp[J, m] * torch.cos(2 * np.pi * g[m])
    del g
    s = ffth.Solver(np.zeros((n, n, n), np.uint16), 3.0, 2.0, lame=lame, order=1, nloads=1)
    P, gmean = s.order1_rhs(eps0, grad.reshape(18))
    assert np.allclose(gmean, gmean_ref, rtol=1e-12, atol=1e-12)
    idx = rng.integers(0, n, size=(3, 2000))
    yc = -0.5 + (idx + 0.5) / n
    yf = -0.5 + (0.5) / nc           # coarse-grid origin offset: y = yf + j/nc
    expect = np.zeros((6, idx.shape[1]))
    for k in ks:
        ksig = np.array([kk if kk < nc // 2 else kk - nc for kk in k])
        ph = np.exp(2j * np.pi * (ksig[:, None] * (yc - yf) * nc).sum(0) / nc)
        expect += np.real(coef[(slice(None),) + k][:, None] * ph)
    got = P[:, idx[0], idx[1], idx[2]].cpu().numpy()
    assert np.abs(got - expect).max() < 1e-11 * np.abs(expect).max()


def test_fibres512_mixed_cg_one_load():
    """512^3 aligned fibres (contrast 1000): the FP32/FP64 CG converges to 1e-8
    and the result is independent of x3 (fibres parallel to x3, load e_1)."""
    torch = require_gpu()
    print("case fibres512", flush=True)
    phase, lame = M.hex_fibres(512)
    lam0, mu0 = M.midpoint_reference(lame)
    s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=1, precision="mixed", tol=1e-8, max_iter=50000)
    eps, res = s.solve_order0([1, 0, 0, 0, 0, 0])
    assert res[0]["status"] == 0 and res[0]["residual"] < 1e-8
    e = eps[0]
    var = (e - e.mean(dim=3, keepdim=True)).abs().max().item()
    assert var < 1e-6 * e.abs().max().item()
    print("fibres512 iters", res[0]["iters"], "outer", res[0]["outer_iters"])
