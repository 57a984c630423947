"""Pins of the oracle's filter bank (Section 2, "Finite Discrete Shearlets", Theorem 2.2,
Remark 2.3) against what the paper fixes: the number of filters, the Parseval identity
sum_j psi_j(w)^2 = 1 at every frequency, the cone and radial supports, symmetry, and
the mirror relation between the two cones."""
import json
import os

import numpy as np
import pytest

from oracle import filter_bank, filter_list, freq_index, num_filters

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
CASES = [(8, 1), (15, 2), (16, 2), (32, 2), (48, 2), (64, 3), (96, 3), (128, 2), (128, 3), (256, 4)]


def test_filter_count():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    assert num_filters(4) == g["eta_for_4_scales"]["value"]       # Remark 2.3: 61 images at 4 scales
    assert [num_filters(J) for J in (1, 2, 3, 4)] == [5, 13, 29, 61]
    for J in (1, 2, 3, 4):
        fl = filter_list(J)
        assert len(fl) == num_filters(J)
        for j in range(J):   # per scale: 2^(j+1)-1 shears per cone plus the two seams k = -+2^j
            assert sum(1 for kind, jj, _ in fl if jj == j and kind == "h") == 2 ** (j + 1) - 1
            assert sorted(k for kind, jj, k in fl if jj == j and kind == "seam") == [-(2 ** j), 2 ** j]


@pytest.mark.parametrize("n,J", CASES)
def test_parseval_every_bin(n, J):
    # Theorem 2.2: the system is a Parseval frame, equivalently sum_j psi_j(w)^2 = 1 for
    # every w in Omega.
    B = filter_bank(n, J)
    assert B.shape == (num_filters(J), n, n)
    assert np.max(np.abs(np.sum(B ** 2, axis=0) - 1.0)) < 1e-13
    assert np.all(B >= 0.0) and np.all(B <= 1.0 + 1e-12)


@pytest.mark.parametrize("n,J", CASES)
def test_symmetry(n, J):
    # psi_j(-w) = psi_j(w) (mod N): the coefficient images of a real image are real.
    B = filter_bank(n, J)
    m = (-np.arange(n)) % n
    assert np.array_equal(B, B[:, m][:, :, m])


@pytest.mark.parametrize("n,J", [(32, 2), (64, 3), (128, 2), (256, 4)])
def test_supports(n, J):
    B = filter_bank(n, J, symmetrize_nyquist=False)
    om = freq_index(n)
    a1 = np.abs(om)[:, None] * np.ones((1, n), dtype=np.int64)
    a2 = np.abs(om)[None, :] * np.ones((n, 1), dtype=np.int64)
    rho = 4.0 ** J / n
    rmax = rho * np.maximum(a1, a2)
    for f, (kind, j, k) in zip(B, filter_list(J)):
        if kind == "low":
            assert f[0, 0] == 1.0
            assert np.all(f[rmax >= 1.0] == 0.0) and np.all(f[rmax <= 0.5] == 1.0)
            continue
        assert f[0, 0] == 0.0
        # radial support of psi1_hat(4^-j .): ||xi||_inf in [4^j/2, 4^(j+1)]
        assert np.all(f[(rmax < 4.0 ** j / 2) | (rmax > 4.0 ** (j + 1))] == 0.0)
        if kind == "h":
            assert np.all(f[a2 >= a1] == 0.0)                     # C^h only
        elif kind == "v":
            assert np.all(f[a1 >= a2] == 0.0)                     # C^v only
        # angular support: |2^j t + k| < 1 with t the slope inside the cone
        with np.errstate(divide="ignore", invalid="ignore"):
            t_h = om[None, :] / np.where(om[:, None] == 0, np.nan, om[:, None])
            t_v = om[:, None] / np.where(om[None, :] == 0, np.nan, om[None, :])
        bad_h = (a2 <= a1) & (np.abs(2.0 ** j * t_h + k) >= 1.0)
        bad_v = (a1 < a2) & (np.abs(2.0 ** j * t_v + k) >= 1.0)
        assert np.all(f[bad_h | bad_v] == 0.0)


@pytest.mark.parametrize("n,J", [(32, 2), (64, 3), (15, 2)])
def test_cone_mirror(n, J):
    # Swapping omega_1 and omega_2 maps the horizontal shearlet (j,k) onto the vertical one
    # (j,k) (the two cone families are defined by the same formula with the roles of the
    # axes exchanged); the glued seam filters map onto themselves.
    B = filter_bank(n, J)
    fl = filter_list(J)
    idx = {f: i for i, f in enumerate(fl)}
    for i, (kind, j, k) in enumerate(fl):
        if kind == "h":
            assert np.array_equal(B[i].T, B[idx[("v", j, k)]])
        if kind in ("seam", "low"):
            assert np.array_equal(B[i].T, B[i])


def test_seam_pairing_is_continuous():
    # The glued seam filter combines the halves of both cones that sit on the same
    # diagonal: for k = +2^j near w2 = -w1 and for k = -2^j near w2 = w1.
    n, J = 64, 3
    B = filter_bank(n, J, symmetrize_nyquist=False)
    fl = filter_list(J)
    om = freq_index(n)
    for i, (kind, j, k) in enumerate(fl):
        if kind != "seam":
            continue
        s = 1 if k < 0 else -1
        # nonzero only near the line w2 = s * w1
        nz = np.argwhere(B[i] > 0)
        w1, w2 = om[nz[:, 0]], om[nz[:, 1]]
        assert np.all(np.abs(w2 - s * w1) < np.maximum(np.abs(w1), np.abs(w2)))


def test_nyquist_reading_needed():
    # Without the even-N Nyquist symmetrisation the coefficient images are complex
    # (the reading documented in the oracle); with it, Parseval still holds bin-wise.
    from oracle import fft2, ifft2
    n, J = 32, 2
    f = np.random.default_rng(3).normal(size=(n, n))
    raw = filter_bank(n, J, symmetrize_nyquist=False)
    im = max(np.max(np.abs(ifft2(b * fft2(f)).imag)) for b in raw)
    assert im > 1e-6
    sym = filter_bank(n, J)
    assert max(np.max(np.abs(ifft2(b * fft2(f)).imag)) for b in sym) < 1e-13
    assert np.max(np.abs(np.sum(raw ** 2, 0) - 1)) < 1e-13
