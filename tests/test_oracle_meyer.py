"""Pins of the oracle's one-dimensional building blocks (Section 2) against the
identities the paper states for them (Lemma 2.1, the scaling-function overlap
identity, the supports shown in Fig. 2) and against elementary closed-form values."""
import numpy as np
import pytest

from oracle import meyer_b, meyer_v, phi_1d, psi1_hat, psi2_hat

X = np.linspace(-3.0, 3.0, 60001)


def test_v_symmetry_identity():
    # v(x) + v(1 - x) = 1 for every x: the property the angular partition rests on.
    assert np.max(np.abs(meyer_v(X) + meyer_v(1.0 - X) - 1.0)) < 1e-13


def test_v_values_and_shape():
    assert meyer_v(0.0) == 0.0 and meyer_v(1.0) == 1.0
    assert meyer_v(0.5) == pytest.approx(0.5, abs=1e-15)
    assert np.all(meyer_v(X[X < 0]) == 0.0) and np.all(meyer_v(X[X > 1]) == 1.0)
    t = np.linspace(0, 1, 10001)
    assert np.all(np.diff(meyer_v(t)) >= -1e-15)             # monotone on [0, 1]
    # C^3 smoothness at the ends: v(x) = O(x^4) at 0 and 1 - v = O((1-x)^4) at 1.
    h = 1e-3
    assert meyer_v(h) < 40 * h ** 4 and 1.0 - meyer_v(1 - h) < 40 * h ** 4


def test_b_dyadic_partition():
    # sum_m b(2^m x)^2 = 1 for every x != 0 (Meyer's partition; gives Lemma 2.1's first part).
    x = np.concatenate([np.linspace(0.01, 40, 20001), -np.linspace(0.01, 40, 2001)])
    tot = sum(meyer_b(2.0 ** m * x) ** 2 for m in range(-12, 12))
    assert np.max(np.abs(tot - 1.0)) < 1e-13
    assert meyer_b(2.0) == pytest.approx(1.0, abs=1e-15)
    assert meyer_b(1.0) == 0.0 and meyer_b(4.0) == pytest.approx(0.0, abs=1e-15)


def test_psi1_support():
    # Fig. 2: supp psi1_hat = [-4, -1/2] u [1/2, 4].
    inside = (np.abs(X) > 0.5) & (np.abs(X) < 4.0)
    assert np.all(psi1_hat(X[~inside]) < 1e-12)
    assert np.all(psi1_hat(X[inside]) > 0.0)
    assert psi1_hat(1.0) == pytest.approx(1.0, abs=1e-15)     # b(2)=1, b(1)=0


def test_psi2_support_and_peak():
    # Fig. 2: supp psi2_hat = [-1, 1]; peak 1 at 0; even.
    assert np.all(psi2_hat(X[np.abs(X) >= 1.0]) == 0.0)
    assert np.all(psi2_hat(X[np.abs(X) < 1.0]) > 0.0)
    assert psi2_hat(0.0) == 1.0
    assert np.max(np.abs(psi2_hat(X) - psi2_hat(-X))) < 1e-15


def test_lemma_2_1_radial():
    # sum_{j>=0} psi1_hat(4^-j w)^2 = 1 for |w| > 1.
    w = np.concatenate([np.linspace(1.0001, 5000, 40001), -np.linspace(1.0001, 300, 3001)])
    tot = sum(psi1_hat(w / 4.0 ** j) ** 2 for j in range(0, 12))
    assert np.max(np.abs(tot - 1.0)) < 1e-13


@pytest.mark.parametrize("j", [0, 1, 2, 3, 4])
def test_lemma_2_1_angular(j):
    # sum_{k=-2^j}^{2^j} psi2_hat(k + 2^j w)^2 = 1 for |w| <= 1.
    w = np.linspace(-1.0, 1.0, 20001)
    tot = sum(psi2_hat(k + 2.0 ** j * w) ** 2 for k in range(-(2 ** j), 2 ** j + 1))
    assert np.max(np.abs(tot - 1.0)) < 1e-13


def test_scaling_overlap_identity():
    # |psi1_hat(w)|^2 + |phi(w)|^2 = 1 on |w| in [1/2, 1]  (eq. (OverlapPsi1_2)),
    # and the piecewise value of sum_j psi1_hat(4^-j w)^2 stated just before it.
    w = np.concatenate([np.linspace(0.5, 1.0, 5001), -np.linspace(0.5, 1.0, 501)])
    assert np.max(np.abs(psi1_hat(w) ** 2 + phi_1d(w) ** 2 - 1.0)) < 1e-13
    t = np.linspace(0.0, 6.0, 60001)
    tot = sum(psi1_hat(t / 4.0 ** j) ** 2 for j in range(0, 8))
    expect = np.where(t <= 0.5, 0.0, np.where(t < 1.0, np.sin(0.5 * np.pi * meyer_v(2 * t - 1)) ** 2, 1.0))
    assert np.max(np.abs(tot - expect)) < 1e-13


def test_phi_profile():
    assert np.all(phi_1d(X[np.abs(X) <= 0.5]) == 1.0)
    assert np.all(phi_1d(X[np.abs(X) >= 1.0]) == 0.0)
    mid = X[(np.abs(X) > 0.5) & (np.abs(X) < 1.0)]
    assert np.all((phi_1d(mid) >= 0) & (phi_1d(mid) <= 1))
    core = X[(np.abs(X) > 0.55) & (np.abs(X) < 0.95)]
    assert np.all((phi_1d(core) > 0) & (phi_1d(core) < 1))
    assert np.all(np.diff(phi_1d(np.linspace(0.5, 1.0, 1001))) <= 1e-15)   # decreasing
