"""Pins of the oracle's DFT pair (Section 2: fft2 / ifft2 and Plancherel) against a
direct evaluation of the defining sums on tiny grids, including odd sizes."""
import numpy as np
import pytest

from oracle import fft2, freq_index, ifft2, naive_dft2


@pytest.mark.parametrize("n", [4, 5, 6, 8, 9, 10, 12, 15, 16])
def test_fft_matches_direct_sum(n):
    rng = np.random.default_rng(n)
    f = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    assert np.max(np.abs(fft2(f) - naive_dft2(f))) < 1e-11
    F = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    assert np.max(np.abs(ifft2(F) - naive_dft2(F, inverse=True))) < 1e-12
    assert np.max(np.abs(ifft2(fft2(f)) - f)) < 1e-13


@pytest.mark.parametrize("n", [7, 8, 32])
def test_plancherel(n):
    # <f, g> = N^-2 <f_hat, g_hat>.
    rng = np.random.default_rng(100 + n)
    f, g = rng.normal(size=(2, n, n))
    lhs = np.sum(f * g)
    rhs = np.vdot(fft2(g), fft2(f)).real / n ** 2
    assert abs(lhs - rhs) < 1e-11 * n * n


@pytest.mark.parametrize("n", [1, 2, 5, 8, 9, 128])
def test_frequency_set(n):
    # Omega = {-floor(N/2), .., ceil(N/2) - 1}, each frequency once, FFT index = omega mod N.
    om = freq_index(n)
    assert sorted(om.tolist()) == list(range(-(n // 2), (n + 1) // 2))
    assert np.all(om % n == np.arange(n))
