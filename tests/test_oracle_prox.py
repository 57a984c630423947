"""Pins of the oracle's proximal maps (Section 3): soft shrinkage against its
defining minimisation, and the pixelwise simplex projection against brute-force
enumeration, the paper's own re-projection procedure, and the KKT conditions."""
import numpy as np
import pytest

from oracle import project_simplex, project_simplex_bruteforce, project_simplex_paper, soft_shrink


def test_shrink_piecewise_and_boundary():
    t = 0.3
    x = np.array([-1.0, -0.3, -0.2, 0.0, 0.2, 0.3, 0.30000001, 2.0])
    assert np.allclose(soft_shrink(x, t), [-0.7, 0.0, 0.0, 0.0, 0.0, 0.0, 1e-8, 1.7], atol=1e-15)
    assert soft_shrink(0.3, 0.3) == 0.0                           # |x| = t -> 0
    assert np.all(soft_shrink(x, 0.0) == x)


def test_shrink_is_prox_of_l1():
    # S_t(x) = argmin_v  t|v| + (v - x)^2 / 2  (the v-update minimisation of Section 3).
    grid = np.linspace(-4, 4, 800001)
    rng = np.random.default_rng(0)
    for x, t in zip(rng.normal(size=25) * 2, rng.uniform(0, 1.5, size=25)):
        obj = t * np.abs(grid) + 0.5 * (grid - x) ** 2
        assert abs(grid[np.argmin(obj)] - soft_shrink(x, t)) < 2e-5


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6])
def test_simplex_vs_bruteforce_and_paper(q):
    rng = np.random.default_rng(q)
    g = rng.normal(size=(q, 400)) * rng.choice([0.1, 1.0, 5.0], size=(1, 400))
    g[:, :5] = 0.25                                   # ties
    p = project_simplex(g)
    assert np.max(np.abs(p - project_simplex_bruteforce(g))) < 1e-13
    assert np.max(np.abs(p - project_simplex_paper(g))) < 1e-13


@pytest.mark.parametrize("q", [2, 3, 5, 8])
def test_simplex_kkt(q):
    rng = np.random.default_rng(10 + q)
    g = rng.normal(size=(q, 2000)) * 2
    x = project_simplex(g)
    assert np.all(x >= 0) and np.max(np.abs(x.sum(0) - 1)) < 1e-14
    # KKT: x = max(g - tau, 0) with one tau per pixel; g_i - tau <= 0 where x_i = 0.
    pos = x > 0
    tau = np.where(pos, g - x, np.nan)
    tmax, tmin = np.nanmax(tau, axis=0), np.nanmin(tau, axis=0)
    assert np.max(tmax - tmin) < 1e-13
    assert np.all(np.where(~pos, g - tmax[None] <= 1e-13, True))
    # order preserving and invariant under adding a constant to all labels
    order = np.argsort(g, axis=0)
    xs = np.take_along_axis(x, order, axis=0)
    assert np.all(np.diff(xs, axis=0) >= -1e-15)
    assert np.max(np.abs(project_simplex(g + 3.7) - x)) < 1e-13


def test_simplex_fixed_points():
    e = np.eye(4)
    assert np.array_equal(project_simplex(e), e)
    x = np.full((4, 1), 0.25)
    assert np.allclose(project_simplex(x), x, atol=1e-16)
