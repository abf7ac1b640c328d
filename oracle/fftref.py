"""Own discrete Fourier transform for the oracle (test infrastructure only).

Convention (the paper fixes only that the Fourier series runs over
xi in (2 pi Z)^d on the unit periodic cell, Sec. 2, eq. (5)):

    forward   F[k] = sum_j f[j] exp(-2 pi i k j / n)
    inverse   f[j] = (1/n) sum_k F[k] exp(+2 pi i k j / n)

so that a gradient becomes multiplication by +i xi with xi = 2 pi k.

Two implementations, kept deliberately plain:
  * ``dft_direct``: the O(n^2) definition as a matrix product;
  * ``fft``: recursive decimation-in-time Cooley-Tukey over the smallest
    prime factor, falling back to the direct DFT for n <= 16 or prime n.
Both transform along one axis of an n-d array; ``fftn3`` / ``ifftn3`` apply
them along the last three axes.
"""
import numpy as np

__all__ = ["dft_direct", "fft", "ifft", "fftn3", "ifftn3", "dft_matrix"]


def dft_matrix(n, sign=-1):
    """n x n matrix W[k, j] = exp(sign * 2 pi i k j / n), exponent reduced mod n."""
    k = np.arange(n)
    kj = np.outer(k, k) % n
    return np.exp(sign * 2j * np.pi * kj / n)


def _smallest_factor(n):
    p = 2
    while p * p <= n:
        if n % p == 0:
            return p
        p += 1
    return n


def _dft_last(x, sign):
    return x @ dft_matrix(x.shape[-1], sign).T


def _fft_last(x, sign):
    """Unnormalised transform along the last axis."""
    n = x.shape[-1]
    p = _smallest_factor(n)
    if n <= 16 or p == n:
        return _dft_last(x, sign)
    m = n // p
    # x[p*j + s] -> subsequence s, element j
    sub = np.moveaxis(x.reshape(x.shape[:-1] + (m, p)), -1, -2)     # [..., s, j]
    y = _fft_last(sub, sign)                                         # [..., s, k2]
    s = np.arange(p)
    k2 = np.arange(m)
    y = y * np.exp(sign * 2j * np.pi * (np.outer(s, k2) % n) / n)    # twiddle w_n^(s k2)
    # X[k1*m + k2] = sum_s w_p^(k1 s) y[s, k2]
    out = np.einsum("qs,...sk->...qk", dft_matrix(p, sign), y)
    return out.reshape(x.shape)


def dft_direct(x, axis=-1, inverse=False):
    """O(n^2) DFT along ``axis`` (the definition; used as the FFT's pin)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    sign = +1 if inverse else -1
    y = _dft_last(x, sign)
    if inverse:
        y = y / x.shape[-1]
    return np.moveaxis(y, -1, axis)


def fft(x, axis=-1):
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last(x, -1), -1, axis)


def ifft(x, axis=-1):
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last(x, +1) / x.shape[-1], -1, axis)


def fftn3(x):
    """Forward 3-D transform over the last three axes."""
    y = fft(x, axis=-1)
    y = fft(y, axis=-2)
    return fft(y, axis=-3)


def ifftn3(x):
    """Inverse 3-D transform (with the 1/(n0 n1 n2) factor) over the last three axes."""
    y = ifft(x, axis=-3)
    y = ifft(y, axis=-2)
    return ifft(y, axis=-1)
