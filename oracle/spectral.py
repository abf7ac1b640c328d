"""Spectral operators of the oracle (test infrastructure only).

Grid convention: the periodic cell is [-1/2, 1/2)^3 (Sec. 2); voxel j along
an axis of n voxels has centre -1/2 + (j + 1/2)/n.  Frequencies use the
signed index k = j for j < n/2, else j - n, and xi = 2 pi k (Sec. 2, the
lattice (2 pi Z)^d of eq. (5)).

Nyquist rule (the paper sums over the infinite lattice and is silent on the
truncation): for an even n_d every mode with k_d = -n_d/2 is set to zero in
the output of every spectral operator here (Green operator, theta, the
displacement recovery, the spectral gradient).  The zero frequency is set to
zero as the paper prescribes for the Green operator (Algorithm 1, the step
after the Green operator) and for theta (defined for xi != 0 only, Sec. 3,
eq. (12)).
"""
import numpy as np

from . import fftref


def frequencies(shape):
    """xi (3, n0, n1, n2) and the mask of retained modes (xi != 0, no Nyquist index)."""
    ks = []
    keep = np.ones(shape, dtype=bool)
    for d, n in enumerate(shape):
        j = np.arange(n)
        k = np.where(j < (n + 1) // 2, j, j - n)         # signed index; for even n, j = n/2 -> -n/2
        shp = [1, 1, 1]
        shp[d] = n
        ks.append(k.reshape(shp).astype(np.float64))
        if n % 2 == 0:
            keep &= (k.reshape(shp) != -n // 2)
    kk = np.broadcast_arrays(*ks)
    xi = 2.0 * np.pi * np.stack(kk)
    keep &= ~((kk[0] == 0) & (kk[1] == 0) & (kk[2] == 0))
    return xi, keep


def gamma0_hat(xi, lam0, mu0):
    """Green operator coefficients for xi != 0 (the formula given below eq. (5)).

    xi: (3, m) -> (3, 3, 3, 3, m), written term by term from the paper:
      (d_ki xi_l xi_j + d_li xi_k xi_j + d_kj xi_l xi_i + d_lj xi_k xi_i) / (4 mu0 |xi|^2)
      - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) * xi_i xi_j xi_k xi_l / |xi|^4
    """
    d = np.eye(3)
    n2 = np.sum(xi * xi, axis=0)
    first = (np.einsum("ki,lm,jm->ijklm", d, xi, xi)
             + np.einsum("li,km,jm->ijklm", d, xi, xi)
             + np.einsum("kj,lm,im->ijklm", d, xi, xi)
             + np.einsum("lj,km,im->ijklm", d, xi, xi)) / (4.0 * mu0 * n2)
    second = np.einsum("im,jm,km,lm->ijklm", xi, xi, xi, xi) / (n2 * n2)
    return first - (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) * second


def green_apply_hat(tau_hat, lam0, mu0):
    """eta_hat = -Gamma0_hat(xi) : tau_hat on retained modes, 0 elsewhere (Algorithm 1)."""
    shape = tau_hat.shape[2:]
    xi, keep = frequencies(shape)
    out = np.zeros_like(tau_hat)
    for i0 in range(shape[0]):                    # one plane at a time bounds memory
        kp = keep[i0]
        if not kp.any():
            continue
        g = gamma0_hat(xi[:, i0][:, kp], lam0, mu0)           # (3,3,3,3,m)
        t = tau_hat[:, :, i0][:, :, kp]                        # (3,3,m)
        out[:, :, i0][:, :, kp] = -np.einsum("ijklm,klm->ijm", g, t)
    return out


def green_apply(tau, lam0, mu0):
    """eta = -(Gamma0 * tau) of eq. (5): real (3,3,n0,n1,n2) field in and out."""
    eta_hat = green_apply_hat(fftref.fftn3(tau), lam0, mu0)
    return np.real(fftref.ifftn3(eta_hat))


def theta_hat_from_g_hat(g_hat):
    """Eq. (12): theta_hat = i/|xi|^4 [ (xi x xi)(g_hat . xi) - (g_hat x xi + xi x g_hat)|xi|^2 ].

    g_hat: (3, n0, n1, n2) -> (3, 3, n0, n1, n2); zero at xi = 0 and Nyquist modes.
    """
    shape = g_hat.shape[1:]
    xi, keep = frequencies(shape)
    n2 = np.sum(xi * xi, axis=0)
    n2 = np.where(keep, n2, 1.0)
    gx = np.sum(g_hat * xi, axis=0)
    outer_xx = np.einsum("i...,j...->ij...", xi, xi)
    sym_gx = np.einsum("i...,j...->ij...", g_hat, xi) + np.einsum("i...,j...->ij...", xi, g_hat)
    th = 1j / (n2 * n2) * (outer_xx * gx - sym_gx * n2)
    return np.where(keep, th, 0.0)


def theta_from_g(g):
    return np.real(fftref.ifftn3(theta_hat_from_g_hat(fftref.fftn3(g))))


def displacement_hat_from_strain_hat(eps_hat):
    """Inverse of eq. (1) in Fourier space for a compatible strain.

    From eps_hat = (i/2)(xi x u_hat + u_hat x xi) one gets
      u_hat = -i [ 2 eps_hat xi / |xi|^2 - xi (xi . eps_hat . xi) / |xi|^4 ],
    with u_hat(0) = 0 (zero-mean displacement, Sec. 2) and Nyquist modes 0.
    """
    shape = eps_hat.shape[2:]
    xi, keep = frequencies(shape)
    n2 = np.where(keep, np.sum(xi * xi, axis=0), 1.0)
    ex = np.einsum("ij...,j...->i...", eps_hat, xi)
    xex = np.sum(ex * xi, axis=0)
    u = -1j * (2.0 * ex / n2 - xi * xex / (n2 * n2))
    return np.where(keep, u, 0.0)


def displacement_from_strain(eps):
    return np.real(fftref.ifftn3(displacement_hat_from_strain_hat(fftref.fftn3(eps))))


def sym_gradient_hat(u_hat):
    """eps_hat = (i/2)(xi x u_hat + u_hat x xi), eq. (1) with grad -> i xi; retained modes only."""
    shape = u_hat.shape[1:]
    xi, keep = frequencies(shape)
    e = 0.5j * (np.einsum("i...,j...->ij...", xi, u_hat) + np.einsum("i...,j...->ij...", u_hat, xi))
    return np.where(keep, e, 0.0)


def sym_gradient(u):
    return np.real(fftref.ifftn3(sym_gradient_hat(fftref.fftn3(u))))
