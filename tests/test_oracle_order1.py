"""Pins of the oracle's order-1 (strain-gradient) right-hand side and solve."""
import numpy as np
import pytest

from oracle import homogenization as H
from oracle import tensors
from paper_1712_05145_amd import microstructure as M

MULT = [1.0, 1.0, 1.0, 2.0, 2.0, 2.0]


def _unit_tensor(J):
    e = np.zeros(6)
    e[J] = 1.0
    return tensors.tensor_from_engineering(e)


def test_order1_homogeneous_material_gives_zero():
    phase = np.zeros((5, 5, 5), dtype=np.uint16)
    prob = H.make_problem(phase, 2.0, 1.0, lame=[[1.0, 0.7]])
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.zeros((6, 3))
    grad[0, 0] = grad[1, 1] = 1.0
    eps2, info = H.solve_order1(prob, corr, grad, "cg", tol=1e-12)
    assert info["iters"] == 0 and np.abs(eps2).max() == 0.0
    # <g> = C : (dE/dY contracted): g_1 = C_11kl dE_kl/dY_1 ...
    c = tensors.isotropic_stiffness(1.0, 0.7)
    gm = np.zeros(3)
    for J in range(6):
        gm += MULT[J] * np.einsum("ij,j->i", np.einsum("ijkl,kl->ij", c, _unit_tensor(J)), grad[J])
    assert np.allclose(info["g_mean"], gm, atol=1e-13)


def test_order1_mean_body_force_equals_effective_stiffness_contraction():
    """<g_i> = sum_J c_J <S^(J)>_ij G_Jj and <S^(J)> is column J of C_eff."""
    phase, lame = M.centred_sphere(8)
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    ceff, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    grad = np.random.default_rng(3).standard_normal((6, 3))
    _, _, _, g, g_mean = H.order1_rhs(prob, corr, grad)
    expect = np.zeros(3)
    for J in range(6):
        s = tensors.field_from_voigt6(ceff[:, J])
        expect += MULT[J] * s @ grad[J]
    assert np.allclose(g_mean, expect, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("n", [7, 9])
def test_order1_laminate_exact_1d_reduction(n):
    """Laminate normal to x3 on an odd grid: the 3-D order-0 correctors, the
    order-1 right-hand side (displacements, p_2, g, theta) and the order-1
    solution all reduce to closed-form 1-D quantities."""
    rng = np.random.default_rng(n)
    layers = rng.integers(0, 3, size=n)
    phase = M.laminate((n, n, n), layers, axis=2)
    lame = M.lame_from_young([1.0, 5.0, 2.5], [0.3, 0.25, 0.35])
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    grad = rng.standard_normal((6, 3))
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-13)
    eps2, info = H.solve_order1(prob, corr, grad, "cg", tol=1e-13)

    # ---- independent 1-D computation ----
    cprof = np.stack([tensors.isotropic_stiffness(*lame[p]) for p in layers])   # (n,3,3,3,3)
    q = cprof[:, :, 2, :, 2]
    qinv = np.linalg.inv(q)
    eps1d, disp1d = [], []
    for J in range(6):
        ej = _unit_tensor(J)
        pz = np.einsum("nikl,kl->ni", cprof[:, :, 2], ej)           # (C:E)_{i3}
        c = np.linalg.solve(qinv.mean(0), np.einsum("nik,nk->i", qinv, pz) / n)
        du = np.einsum("nik,nk->ni", qinv, c[None] - pz)           # u'(x3)
        e = np.zeros((n, 3, 3))
        e[:, :, 2] += 0.5 * du
        e[:, 2, :] += 0.5 * du
        eps1d.append(e)
        disp1d.append(H.antiderivative_1d(du))                      # zero-mean u(x3)
    # order-0 correctors agree
    for J in range(6):
        assert np.abs(np.moveaxis(corr[J][:, :, 0, 0, :], -1, 0) - eps1d[J]).max() < 1e-11
    xg = np.zeros((n, 3, 3))
    g = np.zeros((n, 3))
    for J in range(6):
        xg += MULT[J] * np.einsum("nm,j->nmj", disp1d[J], grad[J])
        s = np.einsum("nijkl,nkl->nij", cprof, eps1d[J] + _unit_tensor(J)[None])
        g += MULT[J] * np.einsum("nij,j->ni", s, grad[J])
    p2 = np.einsum("nijkl,nkl->nij", cprof, 0.5 * (xg + np.swapaxes(xg, 1, 2)))
    F = H.antiderivative_1d(g - g.mean(0))                           # theta_{i3} = F_i
    theta = np.zeros((n, 3, 3))
    theta[:, :, 2] += F
    theta[:, 2, :] += F
    theta[:, 2, 2] -= F[:, 2]
    eps2_1d = H.laminate_1d_solve(cprof, p2 + theta)
    got = np.moveaxis(eps2[:, :, 0, 0, :], -1, 0)
    assert np.abs(got - eps2_1d).max() < 1e-10 * max(1.0, np.abs(eps2_1d).max())
    assert np.allclose(info["g_mean"], g.mean(0), atol=1e-12)
    # the 3-D field is constant in x1, x2
    assert np.abs(eps2 - eps2[:, :, :1, :1, :]).max() < 1e-11


def test_order1_rhs_displacement_from_analytic_correctors():
    """p_2 built from correctors that are symmetric gradients of known displacements."""
    n = 9
    y = -0.5 + (np.arange(n) + 0.5) / n
    g0, g1, g2 = np.meshgrid(y, y, y, indexing="ij")
    rng = np.random.default_rng(4)
    amps = rng.standard_normal((6, 3))
    disp = []
    corr = []
    for J in range(6):
        # u_m = a_Jm sin(2 pi y_{m+1}) -> eps_mm = 2 pi a_Jm cos(2 pi y_{m+1})
        u = np.stack([amps[J, 0] * np.sin(2 * np.pi * g0), amps[J, 1] * np.sin(2 * np.pi * g1),
                      amps[J, 2] * np.sin(2 * np.pi * g2)])
        e = np.zeros((3, 3, n, n, n))
        e[0, 0] = 2 * np.pi * amps[J, 0] * np.cos(2 * np.pi * g0)
        e[1, 1] = 2 * np.pi * amps[J, 1] * np.cos(2 * np.pi * g1)
        e[2, 2] = 2 * np.pi * amps[J, 2] * np.cos(2 * np.pi * g2)
        disp.append(u)
        corr.append(e)
    phase = M.random_phases(n, 2, 1)
    lame = np.array([[1.0, 0.5], [3.0, 2.0]])
    prob = H.make_problem(phase, 2.0, 1.0, lame=lame)
    grad = rng.standard_normal((6, 3))
    _, p2, _, g, _ = H.order1_rhs(prob, corr, grad)
    ref = np.zeros((3, 3, n, n, n))
    for x in np.ndindex(n, n, n):
        m = np.zeros((3, 3))
        for J in range(6):
            for a in range(3):
                for j in range(3):
                    m[a, j] += MULT[J] * disp[J][(a,) + x] * grad[J, j]
        c = tensors.isotropic_stiffness(*lame[phase[x]])
        ref[(slice(None), slice(None)) + x] = np.einsum("ijkl,kl->ij", c, 0.5 * (m + m.T))
    assert np.abs(p2 - ref).max() < 1e-12 * np.abs(ref).max()
