"""Pins of the oracle's stiffness input and of its bound formulas against
results that the mathematics fixes independently of the oracle's own code:

* the 21-coefficient Voigt reading (Sec. 2: C with major and minor
  symmetries, given as an upper-triangular Voigt matrix with engineering
  shear) against the closed-form isotropic tensor, against a uniform
  anisotropic medium (whose effective stiffness is the input itself) and
  against the closed-form laminate of anisotropic layers;
* the Hashin-Shtrikman bulk formula against Hill's exact effective bulk
  modulus of phases with equal shear moduli, where both bounds coincide.
"""
import numpy as np
import pytest

from oracle import homogenization as H
from oracle import tensors
from paper_1712_05145_amd import microstructure as M


def _iso_voigt21(lam, mu):
    """Isotropic Hooke's law written out as a Voigt matrix with engineering
    shear: C11 = C22 = C33 = lam + 2 mu, C12 = C13 = C23 = lam, C44 = C55 =
    C66 = mu (sigma_23 = mu gamma_23), everything else zero."""
    c = np.zeros((6, 6))
    c[:3, :3] = lam
    for a in range(3):
        c[a, a] = lam + 2 * mu
    for a in range(3, 6):
        c[a, a] = mu
    return np.array([c[i, j] for i in range(6) for j in range(i, 6)])


def _random_spd_voigt(rng, k):
    out = []
    for _ in range(k):
        a = rng.standard_normal((6, 6))
        c = a @ a.T + 6 * np.eye(6)
        out.append(c)
    return out


def _upper21(c):
    return np.array([c[i, j] for i in range(6) for j in range(i, 6)])


def test_voigt21_isotropic_reading_equals_lame_tensor():
    """An isotropic phase given as 21 coefficients is the same 4th-order
    tensor as the closed form lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        lam, mu = rng.uniform(0.1, 20.0, 2)
        phase = np.zeros((2, 2, 2), dtype=np.uint16)
        a = tensors.StiffnessField.from_voigt21(phase, _iso_voigt21(lam, mu)[None])
        b = tensors.StiffnessField.from_lame(phase, [[lam, mu]])
        assert np.abs(a.tensors - b.tensors).max() <= 1e-14 * (lam + 2 * mu)


def test_voigt21_isotropic_phases_solve_equals_lame_solve():
    """Fields and effective stiffness of a random two-phase cell are the
    same whether the isotropic phases come as Lame pairs or as 21 Voigt
    coefficients."""
    phase = M.random_phases((6, 5, 7), 2, 8)
    lame = M.lame_from_young([1.0, 8.0], [0.3, 0.22])
    lam0, mu0 = M.midpoint_reference(lame)
    pa = H.make_problem(phase, lam0, mu0, lame=lame)
    pb = H.make_problem(phase, lam0, mu0, voigt21=np.stack([_iso_voigt21(l, m) for l, m in lame]))
    ca, corr_a, _ = H.effective_stiffness(pa, "cg", tol=1e-13)
    cb, corr_b, _ = H.effective_stiffness(pb, "cg", tol=1e-13)
    s = np.abs(ca).max()
    assert np.abs(ca - cb).max() < 1e-11 * s
    for J in range(6):
        assert np.abs(corr_a[J] - corr_b[J]).max() < 1e-10 * max(np.abs(corr_a[J]).max(), 1e-30)


def test_uniform_anisotropic_medium_effective_stiffness_is_input():
    """A uniform medium needs no fluctuation (eps = 0), so column J of the
    effective stiffness, Voigt(<sigma>) under the engineering unit strain
    e_J, is column J of the input Voigt matrix: a wrong shear factor in the
    reading would scale the last three columns."""
    rng = np.random.default_rng(5)
    c66 = _random_spd_voigt(rng, 1)[0]
    phase = np.zeros((4, 6, 5), dtype=np.uint16)
    prob = H.make_problem(phase, 2.0, 1.5, voigt21=_upper21(c66)[None])
    ceff, corr, infos = H.effective_stiffness(prob, "cg", tol=1e-12)
    assert all(np.abs(c).max() < 1e-13 for c in corr)
    assert np.abs(ceff - c66).max() < 1e-13 * np.abs(c66).max()


@pytest.mark.parametrize("layers", [[0, 1, 1, 2, 0, 2, 2, 1, 0], [0, 0, 1, 1, 1, 2, 2]])
def test_anisotropic_laminate_matches_closed_form(layers):
    """Layers of three random (triclinic) phases normal to x3 on an odd
    grid (no Nyquist mode, so the discrete solution is the exact layered
    one): the oracle's effective stiffness equals the closed-form laminate
    average of the input Voigt matrices (engineering shear)."""
    rng = np.random.default_rng(len(layers))
    cs = _random_spd_voigt(rng, 3)
    n3 = len(layers)
    phase = M.laminate((3, 5, n3), layers, axis=2)
    prob = H.make_problem(phase, 4.0, 3.0, voigt21=np.stack([_upper21(c) for c in cs]))
    ceff, _, _ = H.effective_stiffness(prob, "cg", tol=1e-13)
    f = [np.mean(np.asarray(layers) == k) for k in range(3)]
    ref = H.laminate_layers_voigt(cs, f)
    assert np.abs(ceff - ref).max() < 1e-10 * np.abs(ref).max()
    assert np.abs(ref - ref.T).max() < 1e-12 * np.abs(ref).max()


def test_layered_closed_form_reduces_to_backus():
    """For isotropic layers the anisotropic laminate formula and the Backus
    formula (written independently) agree."""
    lame = M.lame_from_young([1.0, 7.0, 3.0], [0.3, 0.2, 0.35])
    f = [0.2, 0.5, 0.3]
    c66 = [tensors.voigt66_from_upper21(_iso_voigt21(l, m)) for l, m in lame]
    a = H.laminate_layers_voigt(c66, f)
    b = H.laminate_backus(lame[:, 0], lame[:, 1], f)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def test_hashin_shtrikman_bulk_equals_hill_for_equal_shear():
    """Phases with one shear modulus mu: under a hydrostatic macro strain,
    equilibrium of sigma = lam tr(eps) I + 2 mu eps with eps = sym grad u
    gives div div sigma = Laplacian((lam + 2 mu) tr eps) = 0, so
    (lam + 2 mu) tr eps is constant and K_eff = <1 / (K + 4 mu / 3)>^-1 -
    4 mu / 3 for any geometry (Hill).  On an odd grid every non-zero
    frequency is kept, so the discrete solution obeys the same identity
    voxel by voxel; both Hashin-Shtrikman bulk bounds equal K_eff."""
    mu = 1.7
    ks = np.array([1.0, 9.0, 4.0])
    lame = np.stack([ks - 2 * mu / 3, np.full(3, mu)], axis=1)
    phase = M.random_phases((9, 7, 11), 3, 21)
    f = np.array([np.mean(phase == k) for k in range(3)])
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0 * 1.3, lame=lame)
    eps, mean, info = H.solve_order0(prob, [1.0, 1.0, 1.0, 0.0, 0.0, 0.0], "cg", tol=1e-13)
    tr = eps[0, 0] + eps[1, 1] + eps[2, 2] + 3.0
    lam_x = lame[phase.astype(int), 0]
    q = (lam_x + 2 * mu) * tr
    assert np.abs(q - q.mean()).max() < 1e-10 * abs(q.mean())
    k_eff = mean[:3].sum() / 9.0
    hill = 1.0 / np.sum(f / (ks + 4 * mu / 3)) - 4 * mu / 3
    lo, hi = H.hashin_shtrikman_bulk(f, ks, lame[:, 1])
    assert abs(k_eff - hill) < 1e-11 * hill
    assert abs(lo - hill) < 1e-13 * hill and abs(hi - hill) < 1e-13 * hill


def test_hashin_shtrikman_bulk_bounds_bracket_unequal_shear():
    """With unequal shear moduli the two bounds separate and bracket the
    bulk measures of a random cell's effective stiffness."""
    phase = M.random_phases((7, 9, 5), 2, 4)
    lame = M.lame_from_young([1.0, 12.0], [0.3, 0.25])
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    ceff, _, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
    f = np.array([np.mean(phase == k) for k in range(2)])
    k = lame[:, 0] + 2 * lame[:, 1] / 3
    lo, hi = H.hashin_shtrikman_bulk(f, k, lame[:, 1])
    kc, ks_ = H.bulk_energy_measures(ceff)
    assert lo < hi
    assert lo * (1 - 1e-9) <= ks_ <= kc <= hi * (1 + 1e-9)
