"""Pins of the oracle's spectral operators (Green operator, theta, displacement)."""
import numpy as np
import pytest

from oracle import fftref, spectral, tensors


def _rand_sym(rng, shape):
    a = rng.standard_normal((3, 3) + shape)
    return 0.5 * (a + np.swapaxes(a, 0, 1))


def test_gamma0_matches_acoustic_tensor_construction():
    """Gamma0_hat(xi):tau = sym(xi x K^-1 (tau xi)), K_ik = C0_ijkl xi_j xi_l.

    Independent construction of the Green operator of an isotropic medium
    (inverse of the acoustic tensor) checked against the closed form used by
    the oracle."""
    rng = np.random.default_rng(1)
    lam0, mu0 = 2.3, 0.7
    c0 = tensors.isotropic_stiffness(lam0, mu0)
    xi = rng.standard_normal((3, 20))
    g = spectral.gamma0_hat(xi, lam0, mu0)
    for m in range(xi.shape[1]):
        x = xi[:, m]
        k = np.einsum("ijkl,j,l->ik", c0, x, x)
        tau = rng.standard_normal((3, 3))
        tau = tau + tau.T
        v = np.linalg.solve(k, tau @ x)
        ref = 0.5 * (np.outer(x, v) + np.outer(v, x))
        got = np.einsum("ijkl,kl->ij", g[..., m], tau)
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_gamma0_symmetries_and_degree_zero():
    rng = np.random.default_rng(2)
    xi = rng.standard_normal((3, 7))
    g = spectral.gamma0_hat(xi, 1.5, 0.8)
    assert np.allclose(g, np.transpose(g, (2, 3, 0, 1, 4)), atol=1e-15)      # major
    assert np.allclose(g, np.transpose(g, (1, 0, 2, 3, 4)), atol=1e-15)      # minor
    assert np.allclose(g, spectral.gamma0_hat(3.7 * xi, 1.5, 0.8), atol=1e-15)
    assert np.allclose(g, spectral.gamma0_hat(-xi, 1.5, 0.8), atol=1e-15)


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 10, 8), (5, 7, 9)])
def test_projection_idempotent_real_zero_mean(shape):
    """P = Gamma0 C0 is a projection; its output is real with zero mean."""
    rng = np.random.default_rng(3)
    lam0, mu0 = 1.2, 0.9
    c0 = tensors.isotropic_stiffness(lam0, mu0)
    tau = _rand_sym(rng, shape)

    def proj(e):
        return -spectral.green_apply(np.einsum("ijkl,kl...->ij...", c0, e), lam0, mu0)

    p1 = proj(tau)
    p2 = proj(p1)
    assert np.abs(p2 - p1).max() < 1e-12 * np.abs(p1).max()
    assert np.abs(p1.mean(axis=(2, 3, 4))).max() < 1e-14
    eta_h = spectral.green_apply_hat(fftref.fftn3(tau), lam0, mu0)
    assert np.abs(np.imag(fftref.ifftn3(eta_h))).max() < 1e-14


def test_projection_keeps_compatible_fields():
    """P(sym grad u) = sym grad u for a trigonometric u without Nyquist modes."""
    rng = np.random.default_rng(4)
    shape = (8, 6, 10)
    lam0, mu0 = 3.0, 1.1
    c0 = tensors.isotropic_stiffness(lam0, mu0)
    y = [spectral.fftref.np.arange(n) for n in shape]
    u = np.zeros((3,) + shape)
    grid = np.meshgrid(*[(-0.5 + (np.arange(n) + 0.5) / n) for n in shape], indexing="ij")
    for m in range(3):
        for _ in range(4):
            k = [rng.integers(-n // 2 + 1, n // 2) for n in shape]
            ph = rng.uniform(0, 2 * np.pi)
            u[m] += rng.standard_normal() * np.cos(2 * np.pi * sum(ki * gi for ki, gi in zip(k, grid)) + ph)
    eps = spectral.sym_gradient(u)
    out = -spectral.green_apply(np.einsum("ijkl,kl...->ij...", c0, eps), lam0, mu0)
    assert np.abs(out - eps).max() < 1e-12 * np.abs(eps).max()
    del y


def test_sym_gradient_analytic():
    """Spectral sym-gradient of u = (sin(2 pi y1), 0, 0) is eps_11 = 2 pi cos(2 pi y1)."""
    n = 9
    y = -0.5 + (np.arange(n) + 0.5) / n
    u = np.zeros((3, n, n, n))
    u[0] = np.sin(2 * np.pi * y)[:, None, None]
    eps = spectral.sym_gradient(u)
    expect = 2 * np.pi * np.cos(2 * np.pi * y)[:, None, None] * np.ones((n, n, n))
    assert np.abs(eps[0, 0] - expect).max() < 1e-12
    assert np.abs(eps[1:, :]).max() < 1e-12 and np.abs(eps[0, 1:]).max() < 1e-12
    # a shear: u_2 = sin(2 pi y1) -> eps_12 = pi cos(2 pi y1)
    u2 = np.zeros((3, n, n, n))
    u2[1] = np.sin(2 * np.pi * y)[:, None, None]
    e2 = spectral.sym_gradient(u2)
    assert np.abs(e2[0, 1] - 0.5 * expect).max() < 1e-12


def test_displacement_recovery_inverts_strain():
    rng = np.random.default_rng(5)
    shape = (8, 10, 6)
    u = rng.standard_normal((3,) + shape)
    eps = spectral.sym_gradient(u)
    u_back = spectral.displacement_from_strain(eps)
    # u_back equals u minus its mean and minus its Nyquist content
    uh = fftref.fftn3(u)
    _, keep = spectral.frequencies(shape)
    u_ref = np.real(fftref.ifftn3(np.where(keep, uh, 0)))
    assert np.abs(u_back - u_ref).max() < 1e-12
    assert np.abs(u_back.mean(axis=(1, 2, 3))).max() < 1e-14


def test_displacement_recovery_analytic():
    """eps_11 = 2 pi cos(2 pi y1) comes from u_1 = sin(2 pi y1) (grad -> +i xi, xi = 2 pi k)."""
    n = 7
    y = -0.5 + (np.arange(n) + 0.5) / n
    eps = np.zeros((3, 3, n, n, n))
    eps[0, 0] = (2 * np.pi * np.cos(2 * np.pi * y))[:, None, None]
    u = spectral.displacement_from_strain(eps)
    assert np.abs(u[0] - np.sin(2 * np.pi * y)[:, None, None]).max() < 1e-12
    assert np.abs(u[1:]).max() < 1e-12


@pytest.mark.parametrize("shape", [(8, 8, 8), (5, 7, 6)])
def test_theta_divergence_identity(shape):
    """div theta = g - <g> (eq. (12): i xi . theta_hat = g_hat for xi != 0); theta is real."""
    rng = np.random.default_rng(6)
    g = rng.standard_normal((3,) + shape)
    th_hat = spectral.theta_hat_from_g_hat(fftref.fftn3(g))
    theta = np.real(fftref.ifftn3(th_hat))
    assert np.abs(np.imag(fftref.ifftn3(th_hat))).max() < 1e-13
    assert np.allclose(theta, np.swapaxes(theta, 0, 1), atol=1e-15)
    xi, keep = spectral.frequencies(shape)
    div_hat = 1j * np.einsum("ij...,j...->i...", fftref.fftn3(theta), xi)
    gh = fftref.fftn3(g)
    assert np.abs(np.where(keep, div_hat - gh, 0)).max() < 1e-11 * np.abs(gh).max()


def test_theta_analytic_1d():
    """g = (0, 0, cos(2 pi y3)) gives theta_33 = sin(2 pi y3)/(2 pi), all else 0."""
    n = 9
    y = -0.5 + (np.arange(n) + 0.5) / n
    g = np.zeros((3, n, n, n))
    g[2] = np.cos(2 * np.pi * y)[None, None, :]
    th = spectral.theta_from_g(g)
    expect = (np.sin(2 * np.pi * y) / (2 * np.pi))[None, None, :]
    assert np.abs(th[2, 2] - expect).max() < 1e-13
    th[2, 2] = 0
    assert np.abs(th).max() < 1e-13
    # transverse force g_1 = cos(2 pi y3): theta_13 = theta_31 = sin(2 pi y3)/(2 pi)
    g1 = np.zeros((3, n, n, n))
    g1[0] = np.cos(2 * np.pi * y)[None, None, :]
    t1 = spectral.theta_from_g(g1)
    assert np.abs(t1[0, 2] - expect).max() < 1e-13 and np.abs(t1[2, 0] - expect).max() < 1e-13
