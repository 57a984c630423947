"""Pins of the oracle's shrinkage denoising S^T S_lambda S (the transform of Section 2,
eq. (wichtig) and its adjoint, with Section 3's soft shrinkage of the coefficients).

Each pin is fixed by something other than the oracle's own composition: Theorem 2.2
(lambda = 0 gives f back), closed forms when every filter but a chosen set is removed
(the output is then a Fourier multiplier sum_j psi_j^2), the zero map when every
threshold exceeds every coefficient, and the explicit frame matrix built without FFTs.
"""
import numpy as np
import pytest

from oracle import denoise, fft2, filter_bank, forward, ifft2, lambda_per_filter, naive_dft2

BIG = 1e30


@pytest.mark.parametrize("n,J", [(16, 2), (33, 2), (64, 3)])
def test_zero_threshold_is_identity(n, J):
    # Theorem 2.2: S^T S = I, and S_0 is the identity
    f = np.random.default_rng(n + J).normal(size=(n, n))
    B = filter_bank(n, J)
    assert np.max(np.abs(denoise(f, B, np.zeros(B.shape[0])) - f)) < 1e-12


@pytest.mark.parametrize("n,J", [(32, 2), (48, 2)])
def test_huge_threshold_is_zero(n, J):
    f = np.random.default_rng(3).normal(size=(n, n))
    B = filter_bank(n, J)
    assert np.max(np.abs(denoise(f, B, np.full(B.shape[0], BIG)))) == 0.0


@pytest.mark.parametrize("n,J", [(32, 2), (40, 2), (64, 3)])
def test_kept_filters_give_their_fourier_multiplier(n, J):
    # With thresholds 0 on a set K of filters and infinite elsewhere, the output is
    # ifft2(sum_{j in K} psi_j^2 fft2 f) (the shrinkage keeps or kills whole filters).
    rng = np.random.default_rng(n)
    f = rng.normal(size=(n, n))
    B = filter_bank(n, J)
    eta = B.shape[0]
    for keep in ([0], [1, 2], list(range(1, eta, 3)), [eta - 1]):
        lam = np.full(eta, BIG)
        lam[keep] = 0.0
        ref = np.real(ifft2(np.sum(B[keep] ** 2, axis=0) * fft2(f)))
        assert np.max(np.abs(denoise(f, B, lam) - ref)) < 1e-12
    # only the low-pass kept (per-scale weights (0, inf, ...)): the phi^2 multiplier
    lam = lambda_per_filter([0.0] + [BIG] * J, J)
    ref = np.real(ifft2(B[0] ** 2 * fft2(f)))
    assert np.max(np.abs(denoise(f, B, lam) - ref)) < 1e-12


def test_frame_matrix_bruteforce():
    # U: rows are the translated frame elements, from the filter spectra by the defining
    # inverse DFT; U^T soft(U f) must equal the oracle's denoising.
    n, J = 8, 1
    B = filter_bank(n, J)
    rows = []
    for b in B:
        psi = naive_dft2(b.astype(np.complex128), inverse=True).real
        for m1 in range(n):
            for m2 in range(n):
                rows.append(np.roll(np.roll(psi, m1, axis=0), m2, axis=1).ravel())
    U = np.array(rows)
    rng = np.random.default_rng(11)
    f = rng.normal(size=(n, n))
    lam = rng.uniform(0.0, 0.4, size=B.shape[0])
    c = U @ f.ravel()
    t = np.repeat(lam, n * n)
    shrunk = np.sign(c) * np.maximum(np.abs(c) - t, 0.0)
    assert np.max(np.abs(U.T @ shrunk - denoise(f, B, lam).ravel())) < 1e-12


def test_shrinkage_contracts_coefficients():
    # Every coefficient moves toward zero by at most its threshold: ||S f - S_lambda S f||_inf
    # <= max lambda, and the denoised image is closer to zero in coefficient energy.
    n, J = 64, 3
    f = np.random.default_rng(5).normal(size=(n, n))
    B = filter_bank(n, J)
    lam = lambda_per_filter([0.0, 0.1, 0.2, 0.3], J)
    d = denoise(f, B, lam)
    assert np.linalg.norm(forward(d, B)) <= np.linalg.norm(forward(f, B)) + 1e-12
    assert np.linalg.norm(d) < np.linalg.norm(f)
