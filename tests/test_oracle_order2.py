"""Pins of the oracle's problem of the paper's order alpha = 3 ("order 2"
here): right-hand side from the order-0 correctors and the 18 order-1
unit-gradient solutions, and its solve."""
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


def _hessian(rng):
    h = rng.standard_normal((6, 3, 3))
    return 0.5 * (h + np.swapaxes(h, 1, 2))      # symmetric in the two derivative indices


def test_order2_homogeneous_material_gives_zero():
    phase = np.zeros((5, 5, 5), dtype=np.uint16)
    prob = H.make_problem(phase, 2.0, 1.0, lame=[[1.0, 0.7]])
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    sols, means = H.order1_unit_solutions(prob, corr)
    assert np.abs(np.array(sols)).max() == 0.0
    hess = _hessian(np.random.default_rng(1))
    eps3, info = H.solve_order2(prob, corr, sols, hess)
    assert info["iters"] == 0 and np.abs(eps3).max() == 0.0


def test_order2_mean_body_force_equals_order1_stress_contraction():
    """<g_i> = sum_{J,j,m} <S_2^(J,j)>_im H[J,j,m], with <S_2^(J,j)> the mean
    stresses that the order-1 solves report (computed there independently)."""
    phase = M.random_phases((6, 5, 7), 2, 3)
    lame = M.lame_from_young([1.0, 6.0], [0.3, 0.3])
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    sols, means = H.order1_unit_solutions(prob, corr)
    hess = _hessian(np.random.default_rng(2))
    _, _, _, _, g_mean = H.order2_rhs(prob, corr, sols, hess)
    expect = np.zeros(3)
    for J in range(6):
        for j in range(3):
            s = tensors.field_from_voigt6(means[J * 3 + j])
            expect += s @ hess[J, j]
    assert np.allclose(g_mean, expect, rtol=1e-8, atol=1e-11)


def _laminate_1d_order0(cprof, n):
    q = cprof[:, :, 2, :, 2]
    qinv = np.linalg.inv(q)
    eps, disp = [], []
    for J in range(6):
        pz = np.einsum("nikl,kl->ni", cprof[:, :, 2], _unit_tensor(J))
        c = np.linalg.solve(qinv.mean(0), np.einsum("nik,nk->i", qinv, pz) / n)
        du = np.einsum("nik,nk->ni", qinv, c[None] - pz)
        e = np.zeros((n, 3, 3))
        e[:, :, 2] += 0.5 * du
        e[:, 2, :] += 0.5 * du
        eps.append(e)
        disp.append(H.antiderivative_1d(du))
    return eps, disp


def _theta_1d(g):
    F = H.antiderivative_1d(g - g.mean(0))
    theta = np.zeros((g.shape[0], 3, 3))
    theta[:, :, 2] += F
    theta[:, 2, :] += F
    theta[:, 2, 2] -= F[:, 2]
    return theta


def _disp_1d(eps):
    du = np.stack([2 * eps[:, 0, 2], 2 * eps[:, 1, 2], eps[:, 2, 2]], axis=1)
    return H.antiderivative_1d(du)


@pytest.mark.parametrize("n", [7])
def test_order2_laminate_exact_1d_reduction(n):
    """Laminate normal to x3 (odd grid): the 3-D order-0 correctors, the 18
    order-1 unit solutions and the order-2 right-hand side and solution equal
    the 1-D closed forms built independently here (antiderivatives and the
    exact 1-D equilibrium solve)."""
    rng = np.random.default_rng(n + 1)
    layers = rng.integers(0, 3, size=n)
    phase = M.laminate((n, n, n), layers, axis=2)
    lame = M.lame_from_young([1.0, 5.0, 2.5], [0.3, 0.25, 0.35])
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    _, corr, _ = H.effective_stiffness(prob, "cg", tol=1e-13)
    sols, _ = H.order1_unit_solutions(prob, corr, tol=1e-13)
    hess = _hessian(rng)
    eps3, info = H.solve_order2(prob, corr, sols, hess, tol=1e-13)

    # ---- independent 1-D chain ----
    cprof = np.stack([tensors.isotropic_stiffness(*lame[p]) for p in layers])
    eps0, x1 = _laminate_1d_order0(cprof, n)
    eye = np.eye(3)
    v = np.zeros((n, 3, 3))
    g3 = np.zeros((n, 3))
    for J in range(6):
        for j in range(3):
            xe = MULT[J] * np.einsum("na,j->naj", x1[J], eye[j])
            p2 = np.einsum("nijkl,nkl->nij", cprof, 0.5 * (xe + np.swapaxes(xe, 1, 2)))
            s1 = np.einsum("nijkl,nkl->nij", cprof, eps0[J] + _unit_tensor(J)[None])
            g2 = MULT[J] * s1[:, :, j]                                   # g for G[J, j] = 1
            e2 = H.laminate_1d_solve(cprof, p2 + _theta_1d(g2))
            got = np.moveaxis(sols[J * 3 + j][:, :, 0, 0, :], -1, 0)
            assert np.abs(got - e2).max() < 1e-10 * max(1.0, np.abs(e2).max())
            w = _disp_1d(e2)
            v += np.einsum("na,m->nam", w, hess[J, j])
            s2 = np.einsum("nijkl,nkl->nij", cprof, e2) + p2
            g3 += np.einsum("nim,m->ni", s2, hess[J, j])
    p3 = np.einsum("nijkl,nkl->nij", cprof, 0.5 * (v + np.swapaxes(v, 1, 2)))
    eps3_1d = H.laminate_1d_solve(cprof, p3 + _theta_1d(g3))
    got = np.moveaxis(eps3[:, :, 0, 0, :], -1, 0)
    assert np.abs(got - eps3_1d).max() < 1e-9 * max(1.0, np.abs(eps3_1d).max())
    assert np.allclose(info["g_mean"], g3.mean(0), atol=1e-11)
    assert np.abs(eps3 - eps3[:, :, :1, :1, :]).max() < 1e-10
