"""Pins of the oracle's own FFT against the DFT definition and external facts."""
import numpy as np
import pytest

from oracle import fftref


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 12, 16, 18, 20, 32, 48, 64, 96, 100])
def test_fft_matches_direct_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    # the definition, written with explicit loops for small n
    if n <= 16:
        ref = np.array([[sum(x[b, j] * np.exp(-2j * np.pi * k * j / n) for j in range(n))
                         for k in range(n)] for b in range(3)])
        assert np.allclose(fftref.dft_direct(x), ref, atol=1e-12, rtol=0)
    assert np.allclose(fftref.fft(x), fftref.dft_direct(x), atol=1e-11 * n, rtol=0)
    assert np.allclose(fftref.ifft(fftref.fft(x)), x, atol=1e-13 * n, rtol=0)


def test_fft_external_crosscheck_numpy():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 12, 10, 16))
    assert np.abs(fftref.fftn3(x) - np.fft.fftn(x, axes=(-3, -2, -1))).max() < 1e-11


def test_parseval_and_roundtrip_3d():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((6, 8, 6, 10))
    xh = fftref.fftn3(x)
    n = 8 * 6 * 10
    assert abs(np.sum(np.abs(xh) ** 2) / n - np.sum(x * x)) < 1e-10 * np.sum(x * x)
    assert np.abs(np.real(fftref.ifftn3(xh)) - x).max() < 1e-13


def test_single_mode_and_real_input_hermitian():
    n = 12
    j = np.arange(n)
    x = np.exp(2j * np.pi * 5 * j / n)        # pure mode k = 5
    y = fftref.fft(x)
    expect = np.zeros(n, complex)
    expect[5] = n
    assert np.allclose(y, expect, atol=1e-12)
    r = np.random.default_rng(0).standard_normal(n)
    yr = fftref.fft(r)
    assert np.allclose(yr[1:], np.conj(yr[1:][::-1]), atol=1e-12)
