"""FFT realisation of the discrete shearlet transform and its adjoint (Section 2,
eq. (wichtig) and the inverse-transform paragraph).  Oracle: test infrastructure only.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

# Threads used by scipy.fft (same pocketfft algorithm as numpy.fft, threaded over the
# batch).  The benchmark's CPU-baseline leg reports this count.
WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))


def fft2(f: np.ndarray) -> np.ndarray:
    """Unnormalised 2-D DFT over the last two axes (the paper's fft2, Section 2)."""
    return scipy.fft.fft2(f, axes=(-2, -1), workers=WORKERS)


def ifft2(F: np.ndarray) -> np.ndarray:
    """Inverse 2-D DFT with the 1/N^2 factor (the paper's ifft2, Section 2)."""
    return scipy.fft.ifft2(F, axes=(-2, -1), workers=WORKERS)


def naive_dft2(f: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Direct O(N^4) evaluation of the DFT pair of Section 2 (pins fft2/ifft2 on tiny grids)."""
    n = f.shape[-1]
    m = np.arange(n)
    sign = 1.0 if inverse else -1.0
    E = np.exp(sign * 2j * np.pi * np.outer(m, m) / n)     # E[w, m] = exp(-+2 pi i w m / N)
    out = np.zeros(f.shape, dtype=np.complex128)
    for w1 in range(n):
        for w2 in range(n):
            out[..., w1, w2] = np.sum(f * E[w1][:, None] * E[w2][None, :], axis=(-2, -1))
    return out / (n * n) if inverse else out


def forward(f: np.ndarray, bank: np.ndarray, check_real: bool = True) -> np.ndarray:
    """S f: coefficient image c_j = ifft2(psi_j * fft2(f)) for every filter j (eq. (wichtig)).

    f is [N][N] real; the result is [eta][N][N] real.  With symmetric filters the
    product is Hermitian, so the inverse DFT is real up to rounding; that is checked."""
    F = fft2(f)
    out = np.empty((bank.shape[0],) + f.shape, dtype=np.float64)
    scale = np.sqrt(np.sum(f * f)) + 1e-300
    for j in range(bank.shape[0]):
        c = ifft2(bank[j] * F)
        if check_real:
            im = np.max(np.abs(c.imag))
            if im > 1e-12 * scale:
                raise AssertionError(f"filter {j}: imaginary part {im:.3e} of S f is not negligible")
        out[j] = c.real
    return out


def adjoint(c: np.ndarray, bank: np.ndarray) -> np.ndarray:
    """S^T c = ifft2(sum_j psi_j * fft2(c_j)) (inverse-transform paragraph of Section 2:
    the spectra of the forward transform are reused, summed over scales and shears, then
    one inverse FFT).  c is [eta][N][N]; the result is [N][N] real."""
    acc = np.zeros(c.shape[-2:], dtype=np.complex128)
    for j in range(bank.shape[0]):
        acc += bank[j] * fft2(c[j])
    return ifft2(acc).real


def denoise(f: np.ndarray, bank: np.ndarray, lam_f) -> np.ndarray:
    """S^T S_lambda S f: the coefficients of eq. (wichtig), Section 3's soft shrinkage
    S_lambda applied to every coefficient of filter j with threshold lam_f[j], then the
    adjoint of the inverse-transform paragraph.  f [N][N] real, lam_f [eta] >= 0."""
    from .prox import soft_shrink
    c = forward(f, bank)
    return adjoint(soft_shrink(c, np.asarray(lam_f, dtype=np.float64)[:, None, None]), bank)
