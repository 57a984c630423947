"""Pins of the oracle's shearlet transform S and adjoint S^T (Section 2, eq. (wichtig),
Theorem 2.2, the Parseval-frame relations (trafo), the inverse-transform paragraph,
and the translation invariance claimed in the abstract / Section 1)."""
import numpy as np
import pytest

from oracle import adjoint, filter_bank, filter_list, forward, naive_dft2

CASES = [(16, 2), (32, 2), (33, 2), (48, 2), (64, 3), (128, 2)]


def _frame_matrix(n, J):
    """Rows = frame elements psi_{j,m}, built from their spectra
    psi_j(w) exp(-2 pi i <w, m>/N) by the defining inverse DFT (no FFT involved):
    psi_{j,m}(x) = psi_j(x - m) circularly."""
    B = filter_bank(n, J)
    rows = []
    for b in B:
        psi = naive_dft2(b.astype(np.complex128), inverse=True)
        assert np.max(np.abs(psi.imag)) < 1e-13
        psi = psi.real
        for m1 in range(n):
            for m2 in range(n):
                rows.append(np.roll(np.roll(psi, m1, axis=0), m2, axis=1).ravel())
    return np.array(rows), B


@pytest.mark.parametrize("n,J", [(8, 1), (16, 2)])
def test_explicit_frame_matrix(n, J):
    U, B = _frame_matrix(n, J)
    eta = B.shape[0]
    assert U.shape == (eta * n * n, n * n)
    # Parseval frame: U^T U = I_n, and U U^T != I (not a basis), full rank.
    assert np.max(np.abs(U.T @ U - np.eye(n * n))) < 1e-13
    assert np.linalg.matrix_rank(U) == n * n
    assert np.max(np.abs(U @ U.T - np.eye(eta * n * n))) > 0.5
    # eq. (wichtig): <f, psi_{j,m}> equals ifft2(psi_j fft2 f)(m).
    f = np.random.default_rng(1).normal(size=(n, n))
    assert np.max(np.abs(U @ f.ravel() - forward(f, B).ravel())) < 1e-13
    # (trafo): f = U^T (coefficients); and S^T matches U^T on arbitrary coefficients.
    c = np.random.default_rng(2).normal(size=(eta, n, n))
    assert np.max(np.abs(U.T @ c.ravel() - adjoint(c, B).ravel())) < 1e-12


@pytest.mark.parametrize("n,J", CASES)
def test_parseval_reconstruction_adjointness(n, J):
    rng = np.random.default_rng(n * 10 + J)
    B = filter_bank(n, J)
    f = rng.normal(size=(n, n))
    c = forward(f, B)
    assert c.shape == (B.shape[0], n, n)
    assert abs(np.linalg.norm(c) / np.linalg.norm(f) - 1.0) < 1e-13      # ||S f|| = ||f||
    assert np.max(np.abs(adjoint(c, B) - f)) < 1e-12                       # S^T S = I
    d = rng.normal(size=c.shape)
    assert abs(np.sum(c * d) - np.sum(f * adjoint(d, B))) < 1e-10 * np.linalg.norm(d)


@pytest.mark.parametrize("n,J", [(32, 2), (33, 2), (64, 3)])
def test_translation_invariance(n, J):
    # Translating the image translates every coefficient image (no down-sampling).
    B = filter_bank(n, J)
    f = np.random.default_rng(7).normal(size=(n, n))
    sh = (5, -3)
    a = forward(np.roll(f, sh, axis=(0, 1)), B)
    b = np.roll(forward(f, B), sh, axis=(1, 2))
    assert np.max(np.abs(a - b)) < 1e-12


def test_constant_image_only_lowpass():
    n, J = 32, 2
    B = filter_bank(n, J)
    c = forward(np.full((n, n), 0.7), B)
    assert np.max(np.abs(c[0] - 0.7)) < 1e-14
    assert np.max(np.abs(c[1:])) < 1e-14


@pytest.mark.parametrize("n,J", [(32, 2), (64, 3)])
def test_transpose_swaps_cones(n, J):
    B = filter_bank(n, J)
    fl = filter_list(J)
    idx = {f: i for i, f in enumerate(fl)}
    f = np.random.default_rng(9).normal(size=(n, n))
    cf = forward(f, B)
    ct = forward(f.T.copy(), B)
    for i, (kind, j, k) in enumerate(fl):
        other = idx[("v", j, k)] if kind == "h" else idx[("h", j, k)] if kind == "v" else i
        assert np.max(np.abs(ct[i] - cf[other].T)) < 1e-12
