"""Pins of the oracle's nonlocal (NL-means graph) regulariser of Section 4 and its
primal-dual solver: patch distances against the definition, the graph against a
brute-force replay of the paper's sequential selection, structural properties (symmetry,
degree <= 2m, window), adjointness and norm bound of D, and the solver's limits, first
iterate and weak duality."""
import numpy as np
import pytest

from oracle import (apply_D, apply_Dt, datacost, gaussian_patch, nl_energy, nl_graph, nl_primal_dual, nl_tv,
                    patch_distance, project_simplex, window_distances)
from synth import make_small


def _img(n=16, seed=3, C=1):
    w = make_small(n, 3, 1, channels=C, seed=seed, noise=0.1, iters=1)
    return w


def test_gaussian_patch():
    G = gaussian_patch(5, 2.0)
    assert abs(np.sum(G) - 1.0) < 1e-15 and np.allclose(G, G.T) and np.allclose(G, G[::-1])
    assert np.argmax(G) == 12
    assert abs(G[2, 3] / G[2, 2] - np.exp(-1 / 8)) < 1e-14


@pytest.mark.parametrize("C", [1, 3])
def test_window_distances_match_definition(C):
    img = _img(C=C).img
    offs, D = window_distances(img, 5, 15, 2.0)
    assert len(offs) == 224
    G = gaussian_patch(5, 2.0)
    rng = np.random.default_rng(C)
    n = img.shape[-1]
    for _ in range(40):
        k = rng.integers(len(offs))
        r, c = rng.integers(n, size=2)
        j = ((r + offs[k][0]) % n, (c + offs[k][1]) % n)
        ref = patch_distance(img, (r, c), j, G)
        assert abs(D[k, r, c] - ref) <= 1e-14 * ref


def _replay(img, p, window, a, m):
    """Brute-force replay of the selection: every distance by the definition."""
    n = img.shape[-1]
    G = gaussian_patch(p, a)
    rr = (window - 1) // 2
    nbrs = [[] for _ in range(n * n)]
    for i in range(n * n):
        r0, c0 = divmod(i, n)
        k = min(m, 2 * m - len(nbrs[i]))
        if k <= 0:
            continue
        cand = []
        for o1 in range(-rr, rr + 1):
            for o2 in range(-rr, rr + 1):
                j = ((r0 + o1) % n) * n + (c0 + o2) % n
                if j == i or j in nbrs[i] or len(nbrs[j]) >= 2 * m:
                    continue
                cand.append((patch_distance(img, (r0, c0), divmod(j, n), G), j))
        cand.sort()
        for _, j in cand[:k]:
            nbrs[i].append(j)
            nbrs[j].append(i)
    return nbrs


def test_graph_matches_bruteforce_replay_and_structure():
    n, m = 16, 5
    img = _img(n).img
    nbr = nl_graph(img, 5, 15, 2.0, m)
    ref = _replay(img, 5, 15, 2.0, m)
    flat = nbr.reshape(2 * m, -1)
    for i in range(n * n):
        got = [int(j) for j in flat[:, i] if j >= 0]
        assert got == ref[i]
        assert i not in got and len(set(got)) == len(got) and len(got) <= 2 * m
        for j in got:                                   # symmetric weights
            assert i in list(flat[:, j])
        for j in got:                                   # inside the window (periodic)
            dr = min((j // n - i // n) % n, (i // n - j // n) % n)
            dc = min((j % n - i % n) % n, (i % n - j % n) % n)
            assert dr <= 7 and dc <= 7
    # every pixel got at least its own picks unless the window ran out of eligible pixels
    assert np.min(np.sum(flat >= 0, axis=0)) >= m


def test_D_adjoint_kernel_and_norm():
    n, m = 16, 5
    nbr = nl_graph(_img(n, seed=5).img, 5, 15, 2.0, m)
    rng = np.random.default_rng(1)
    u = rng.normal(size=(n, n))
    y = rng.normal(size=(2 * m, n, n))
    assert abs(np.sum(apply_D(u, nbr) * y) - np.sum(u * apply_Dt(y, nbr))) < 1e-11
    assert np.max(np.abs(apply_D(np.full((n, n), 1.7), nbr))) == 0.0
    # power iteration for ||D||^2 <= 4 * max degree
    x = rng.normal(size=(n, n))
    for _ in range(300):
        x = apply_Dt(apply_D(x, nbr), nbr)
        x /= np.linalg.norm(x)
    L2 = np.sum(apply_D(x, nbr) ** 2)
    deg = np.max(np.sum(nbr.reshape(2 * m, -1) >= 0, axis=0))
    assert L2 <= 4 * deg + 1e-9


def test_nl_primal_dual_limits_and_duality():
    n, m = 16, 5
    w = _img(n, seed=7)
    nbr = nl_graph(w.img, 5, 15, 2.0, m)
    s = datacost(w.img, w.codebook)
    q = s.shape[0]
    # first iterate: u^1 = P_C(-tau s) (y^1 = clip of sigma K 0 = 0)
    r1 = nl_primal_dual(s, nbr, 0.1, 0.05, 0.5, 1)
    assert np.max(np.abs(r1.u - project_simplex(-0.05 * s))) < 1e-14 and np.max(np.abs(r1.y)) == 0.0
    # lambda = 0 with a large primal step: the pointwise argmin vertex
    r0 = nl_primal_dual(s, nbr, 0.0, 1e4, 1e-6, 2)
    assert np.array_equal(r0.labels, np.argmin(s, axis=0).astype(np.int32))
    # q = 1
    assert np.max(np.abs(nl_primal_dual(s[:1], nbr, 0.1, 0.1, 0.1, 3).u - 1.0)) < 1e-12
    # weak duality and decay of the gap: D(y) = sum_pixels min_k (s + K^T y)_k
    lam = 0.05
    tau = sigma = 1.0 / np.sqrt(40.0)
    gaps = []
    for K in (5, 50, 400):
        r = nl_primal_dual(s, nbr, lam, tau, sigma, K)
        kty = np.stack([apply_Dt(r.y[l], nbr) for l in range(q)])
        dual = float(np.sum(np.min(s + kty, axis=0)))
        gaps.append(nl_energy(r.u, s, nbr, lam) - dual)
    assert min(gaps) >= -1e-10 and gaps[2] < 0.1 * gaps[0]
    assert nl_tv(r.u, nbr) >= 0.0


def test_planted_mistakes_are_caught():
    import inspect
    import textwrap
    import oracle.nlmodel as NM

    def mutated(fn, old, new):
        src = textwrap.dedent(inspect.getsource(getattr(NM, fn)))
        assert old in src
        ns = dict(vars(NM))
        exec(compile(src.replace(old, new), f"<mutant {fn}>", "exec"), ns)
        return ns[fn]

    n, m = 16, 5
    img = _img(n).img
    # (1) always picking m neighbours ignores the 2m cap: some pixel gets more than 2m
    #     weights or the graph differs from the replay
    bad = mutated("nl_graph", "k = min(m, 2 * m - l)", "k = m")
    try:
        g_bad = bad(img, 5, 15, 2.0, m)
    except IndexError:            # more than 2m neighbours do not fit in D's 2m blocks
        g_bad = None
    assert g_bad is None or not np.array_equal(g_bad, nl_graph(img, 5, 15, 2.0, m))
    # (2) a transpose without the diagonal term breaks adjointness
    bad = mutated("apply_Dt", "        out[ok] -= yy[b][ok]\n", "")
    nbr = nl_graph(img, 5, 15, 2.0, m)
    rng = np.random.default_rng(2)
    u, y = rng.normal(size=(n, n)), rng.normal(size=(2 * m, n, n))
    assert abs(np.sum(apply_D(u, nbr) * y) - np.sum(u * bad(y, nbr))) > 1e-3
