"""Pins of the oracle's primal-dual iteration for the segmentation model (Section 3's
functional; Chambolle & Pock's method, named at the end of Section 3 as the alternative
to the ADMM).

Fixed by things other than the iteration itself: the closed-form first iterates, weak
duality (P(u) >= D(y) for every feasible pair, which needs K^T to be the adjoint of K),
convergence of the gap to zero, the same optimal value as the (separately pinned) ADMM
oracle, the saddle-point fixed-point equations, lambda = 0 (pointwise argmin) and q = 1.
"""
import numpy as np
import pytest

from oracle import (admm, dual_value, energy, filter_bank, forward, lambda_per_filter, primal_dual,
                    project_simplex_bruteforce)
from synth import make_small


def _problem(n=16, q=3, J=1, lam=0.05, seed=2):
    w = make_small(n, q, J, seed=seed, lam=lam, iters=1)
    from oracle import datacost
    s = datacost(w.img, w.codebook)
    B = filter_bank(n, J)
    return s, B, lambda_per_filter(w.lam, J)


def test_first_iterates_closed_form():
    s, B, lam = _problem()
    tau, sigma = 0.7, 0.9
    # y^1 = clip(sigma K 0) = 0, u^1 = P_C(-tau s), ubar^1 = 2 u^1
    r1 = primal_dual(s, B, lam, tau, sigma, 1)
    u1 = np.stack([project_simplex_bruteforce(v) for v in (-tau * s).reshape(s.shape[0], -1).T]).T.reshape(s.shape)
    assert np.max(np.abs(r1.y)) == 0.0
    assert np.max(np.abs(r1.u - u1)) < 1e-12
    assert np.max(np.abs(r1.ubar - 2 * u1)) < 1e-12
    # y^2 = clip(sigma S (2 u^1), +-lambda)
    r2 = primal_dual(s, B, lam, tau, sigma, 2)
    for l in range(s.shape[0]):
        ref = np.clip(sigma * forward(2 * u1[l], B), -lam[:, None, None], lam[:, None, None])
        assert np.max(np.abs(r2.y[l] - ref)) < 1e-12


def test_weak_duality_and_gap_to_zero():
    s, B, lam = _problem()
    r = primal_dual(s, B, lam, 0.9, 0.9, 600, with_gap=True)
    assert np.all(r.gap >= -1e-10)
    p = energy(r.u, s, B, lam)
    # the gap decays like 1/n (the method's rate): 0.89 P at n=6, 1.7e-3 P at n=600
    assert r.gap[-1] < 3e-3 * abs(p)
    assert r.gap[-1] < 0.01 * r.gap[5]
    assert r.gap[50] > r.gap[200] > r.gap[-1]


def test_same_optimum_as_admm():
    s, B, lam = _problem()
    pd = primal_dual(s, B, lam, 0.9, 0.9, 1500)
    ad = admm(s, B, lam, 1.0, 1500)
    e_pd, e_ad = energy(pd.u, s, B, lam), energy(ad.w, s, B, lam)
    assert abs(e_pd - e_ad) < 1e-6 * abs(e_ad)
    # the dual value of the PD iterate certifies both: D(y) <= min <= E
    d = dual_value(pd.y, s, B)
    assert d <= min(e_pd, e_ad) + 1e-10


def test_saddle_point_equations_at_convergence():
    s, B, lam = _problem(seed=5)
    tau, sigma = 0.8, 1.0
    r = primal_dual(s, B, lam, tau, sigma, 2000)
    from oracle import adjoint, project_simplex
    kty = np.stack([adjoint(r.y[l], B) for l in range(s.shape[0])])
    assert np.max(np.abs(project_simplex(r.u - tau * (kty + s)) - r.u)) < 1e-4
    for l in range(s.shape[0]):
        y_fix = np.clip(r.y[l] + sigma * forward(r.u[l], B), -lam[:, None, None], lam[:, None, None])
        assert np.max(np.abs(y_fix - r.y[l])) < 1e-4


def test_lambda_zero_and_single_label():
    s, B, lam = _problem()
    # lambda = 0: y stays 0 and u^1 = P_C(-tau s) is the vertex of the smallest entry
    # once tau separates the two smallest entries by more than 1
    tau = 1e4
    r = primal_dual(s, B, np.zeros_like(lam), tau, 1.0 / tau, 3)
    assert np.array_equal(r.labels, np.argmin(s, axis=0).astype(np.int32))
    assert np.max(np.abs(np.sum(r.u, axis=0) - 1.0)) < 1e-12
    s1 = s[:1]
    r1 = primal_dual(s1, B, lam, 0.9, 0.9, 5)
    assert np.max(np.abs(r1.u - 1.0)) < 1e-12


@pytest.mark.parametrize("n,J", [(24, 2), (33, 2)])
def test_iterates_feasible_and_dual_in_box(n, J):
    s, B, lam = _problem(n=n, J=J, q=4, lam=0.1, seed=n)
    r = primal_dual(s, B, lam, 1.0, 1.0, 20)
    assert np.min(r.u) >= 0.0 and np.max(np.abs(np.sum(r.u, axis=0) - 1.0)) < 1e-12
    assert np.all(np.abs(r.y) <= lam[None, :, None, None] + 1e-15)


def test_planted_mistakes_are_caught():
    import inspect
    import textwrap
    import oracle.primaldual as PD

    def mutated(old, new):
        src = textwrap.dedent(inspect.getsource(PD.primal_dual))
        assert old in src
        ns = dict(vars(PD))
        exec(compile(src.replace(old, new), "<mutant primal_dual>", "exec"), ns)
        return ns["primal_dual"]

    s, B, lam = _problem()
    # (1) a sign error on K^T y: the first iterates still match, but the gap grows instead
    # of shrinking (the convergence pin fails)
    bad = mutated("u - tau * (kty + s)", "u - tau * (s - kty)")
    g = bad(s, B, lam, 0.9, 0.9, 40, with_gap=True).gap
    assert g[-1] > g[5]
    # (2) the clip bound taken without the weights (a dropped lambda_j) leaves the box
    bad = mutated("np.clip(y[l] + sigma * c, -lam, lam)", "np.clip(y[l] + sigma * c, -1.0, 1.0)")
    r = bad(s, B, lam, 0.9, 0.9, 30)
    assert np.max(np.abs(r.y) - lam[None, :, None, None]) > 1e-6
    # (3) no extrapolation (ubar = u^{n+1}): the closed-form second iterate differs
    bad = mutated("ubar = 2.0 * u_new - u", "ubar = u_new")
    ref = primal_dual(s, B, lam, 0.7, 0.9, 2)
    assert np.max(np.abs(bad(s, B, lam, 0.7, 0.9, 2).y - ref.y)) > 1e-6
