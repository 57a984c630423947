"""Pins of the oracle's TV comparison model (Section 4) and its ADMM: adjointness of the
periodic forward-difference gradient, the FFT solve against the explicit stencil, the
isotropic shrinkage against its optimality conditions, closed-form TV values, and the
ADMM's lambda = 0 / q = 1 limits, He-Yuan monotone residual and energy bound."""
import numpy as np
import pytest

from oracle import (datacost, grad, grad_adjoint, group_shrink, labels_of, solve_identity_plus_laplacian, tv,
                    tv_admm, tv_energy)
from synth import make_small


@pytest.mark.parametrize("n", [8, 15, 32])
def test_gradient_adjoint_and_kernel(n):
    rng = np.random.default_rng(n)
    u = rng.normal(size=(3, n, n))
    p = rng.normal(size=(3, 2, n, n))
    assert abs(np.sum(grad(u) * p) - np.sum(u * grad_adjoint(p))) < 1e-11 * np.linalg.norm(p) * np.linalg.norm(u)
    assert np.max(np.abs(grad(np.full((n, n), 2.5)))) == 0.0
    # explicit stencil: grad^T grad u = 4u - (4 neighbours)
    lap = 4 * u[0] - sum(np.roll(u[0], sh, axis=ax) for sh in (1, -1) for ax in (0, 1))
    assert np.max(np.abs(grad_adjoint(grad(u[0])) - lap)) < 1e-12


@pytest.mark.parametrize("n", [8, 17, 64])
def test_fft_solve_inverts_the_stencil(n):
    u = np.random.default_rng(n).normal(size=(n, n))
    r = u + grad_adjoint(grad(u))
    assert np.max(np.abs(solve_identity_plus_laplacian(r) - u)) < 1e-12


def test_group_shrinkage_optimality():
    rng = np.random.default_rng(4)
    g = rng.normal(size=(3, 2, 16, 16))
    t = 1.3
    x = group_shrink(g, t)
    nx = np.sqrt(np.sum(x * x, axis=(0, 1)))
    ng = np.sqrt(np.sum(g * g, axis=(0, 1)))
    on = nx > 0
    # nonzero: g - x = t x / ||x|| (the subgradient of t||x||); zero exactly when ||g|| <= t
    assert np.max(np.abs((g - x - t * x / np.where(on, nx, 1.0)[None, None])[:, :, on])) < 1e-12
    assert np.array_equal(~on, ng <= t)
    assert np.max(np.abs(group_shrink(g, 0.0) - g)) == 0.0
    # the prox value beats random nearby points
    f = lambda z: t * np.sqrt(np.sum(z * z, axis=(0, 1))) + 0.5 * np.sum((z - g) ** 2, axis=(0, 1))
    for _ in range(20):
        assert np.all(f(x) <= f(x + 1e-3 * rng.normal(size=x.shape)) + 1e-15)


def test_tv_closed_forms():
    n = 32
    u = np.zeros((1, n, n))
    u[0, 5:17, :] = 1.0          # a horizontal band: two jumps of 1 per column
    assert abs(tv(u) - 2 * n) < 1e-12
    u2 = np.concatenate([u, 1 - u])   # complementary labels: gradient vectors (g, -g)
    assert abs(tv(u2) - 2 * np.sqrt(2) * n) < 1e-9
    assert tv(np.full((2, n, n), 0.5)) == 0.0
    assert abs(tv(np.roll(u2, (3, 7), axis=(1, 2))) - tv(u2)) < 1e-9


def _problem(n=24, q=3, seed=1, lam=0.2):
    w = make_small(n, q, 1, seed=seed, lam=lam, iters=1)
    return datacost(w.img, w.codebook), lam


def test_tv_admm_limits():
    s, _ = _problem()
    # lambda = 0: the minimiser is the pointwise argmin vertex; the ADMM approaches it
    # slowly where the two smallest costs nearly tie, so check the pixels with a clear gap
    r = tv_admm(s, 0.0, 1.0, 300)
    srt = np.sort(s, axis=0)
    clear = (srt[1] - srt[0]) > 0.05
    assert np.array_equal(r.labels[clear], np.argmin(s, axis=0)[clear])
    assert np.sum(r.w * s) - np.sum(srt[0]) < 0.05 * np.sum(srt[0])
    # q = 1: the simplex is the point 1
    r1 = tv_admm(s[:1], 0.2, 1.0, 5)
    assert np.max(np.abs(r1.w - 1.0)) < 1e-12


def test_tv_admm_residual_monotone_and_energy():
    s, lam = _problem(seed=3)
    r = tv_admm(s, lam, 1.0, 200)
    assert np.all(np.diff(r.r_combined) <= 1e-10 * r.r_combined[0])
    onehot = (np.argmin(s, axis=0)[None] == np.arange(s.shape[0])[:, None, None]).astype(float)
    assert tv_energy(r.w, s, lam) < tv_energy(onehot, s, lam)
    # surrogate approaches the exact energy of w
    assert abs(r.surrogate[-1] - tv_energy(r.w, s, lam)) < 1e-3 * tv_energy(r.w, s, lam)


def test_planted_mistakes_are_caught():
    import inspect
    import textwrap
    import oracle.tvmodel as T

    def mutated(fn, old, new):
        src = textwrap.dedent(inspect.getsource(getattr(T, fn)))
        assert old in src
        ns = dict(vars(T))
        exec(compile(src.replace(old, new), f"<mutant {fn}>", "exec"), ns)
        return ns[fn]

    rng = np.random.default_rng(9)
    u = rng.normal(size=(2, 12, 12))
    p = rng.normal(size=(2, 2, 12, 12))
    # (1) the adjoint shifted the wrong way
    bad = mutated("grad_adjoint", "np.roll(p[..., 0, :, :], 1, axis=-2)", "np.roll(p[..., 0, :, :], -1, axis=-2)")
    assert abs(np.sum(grad(u) * p) - np.sum(u * bad(p))) > 1e-3
    # (2) a shrinkage that removes only half the threshold violates the prox's optimality
    bad = mutated("group_shrink", "1.0 - t / np.where", "1.0 - 0.5 * t / np.where")
    g = rng.normal(size=(2, 2, 8, 8))
    x = bad(g, 0.7)
    nx = np.sqrt(np.sum(x * x, axis=(0, 1)))
    on = nx > 0
    assert np.max(np.abs((g - x - 0.7 * x / np.where(on, nx, 1.0)[None, None])[:, :, on])) > 1e-3
    # (3) a missing identity in the u-solve breaks the inverse
    bad = mutated("solve_identity_plus_laplacian", "(1.0 + e[:, None] + e[None, :])",
                  "(1e-12 + e[:, None] + e[None, :])")
    r = u[0] + grad_adjoint(grad(u[0]))
    assert np.max(np.abs(bad(r) - u[0])) > 1e-3
