"""Pins of the oracle's segmentation model and ADMM (Section 3) against what the
mathematics fixes: optimality of every sub-step, special cases with known answers
(lambda = 0, q = 1), exact invariances (scaling, label permutation, transposition,
circular shift, restart), the non-increasing combined residual of ADMM, and the
paper's RGB data term on its printed codebook."""
import json
import os

import numpy as np
import pytest

import oracle as O
from synth import make_small

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _problem(n=32, q=3, J=2, seed=0, lam=0.1, gamma=1.0, channels=1):
    w = make_small(n, q, J, channels=channels, seed=seed, lam=lam, gamma=gamma)
    s = O.datacost(w.img, w.codebook)
    B = O.filter_bank(n, J)
    lam_f = O.lambda_per_filter(w.lam, J)
    return s, B, lam_f, w


def test_datacost_gray_and_rgb():
    with open(GOLDEN) as fh:
        cb = np.array(json.load(fh)["fish_codebook_rgb_by_label"]["value"])   # [4][3]
    n = 6
    rng = np.random.default_rng(0)
    lab = rng.integers(0, 4, size=(n, n))
    img = np.transpose(cb[lab], (2, 0, 1))                  # pixels exactly on codebook colours
    s = O.datacost(img, cb)
    assert s.shape == (4, n, n)
    assert np.all(np.take_along_axis(s, lab[None], 0) == 0.0)
    k = 2
    assert np.allclose(s[k], np.sum((img - cb[k][:, None, None]) ** 2, axis=0))
    g = rng.uniform(size=(1, n, n))
    assert np.allclose(O.datacost(g, np.array([[0.25], [0.5]]))[1], (g[0] - 0.5) ** 2)
    assert np.allclose(O.datacost(g, np.array([[0.25]]), p=1)[0], np.abs(g[0] - 0.25))


def test_lambda_expansion():
    lam = [0.0, 1.0, 2.0]
    lf = O.lambda_per_filter(lam, 2)
    fl = O.filter_list(2)
    for v, (kind, j, _) in zip(lf, fl):
        assert v == (0.0 if kind == "low" else lam[j + 1])
    per = np.arange(13.0)
    assert np.array_equal(O.lambda_per_filter(per, 2), per)
    with pytest.raises(ValueError):
        O.lambda_per_filter([1.0, 2.0], 2)


def test_first_iterate_closed_form():
    # From the zero state: u^1 = -gamma s / 2, v^1 = S_{gamma Lambda}(S u^1), w^1 = P_C(u^1).
    s, B, lam_f, w = _problem()
    r = O.admm(s, B, lam_f, w.gamma, 1)
    assert np.max(np.abs(r.u + 0.5 * w.gamma * s)) < 1e-15
    for l in range(s.shape[0]):
        Su = O.forward(r.u[l], B)
        assert np.max(np.abs(r.v[l] - O.soft_shrink(Su, w.gamma * lam_f[:, None, None]))) < 1e-14
    assert np.max(np.abs(r.w - O.project_simplex(r.u))) < 1e-15


def test_u_update_is_stationary_point():
    # u^{i+1} zeroes the gradient s + (1/gamma) A^T (A u + b - y) of the quadratic of the
    # u-step, with A = [I (x) S; I].
    s, B, lam_f, w = _problem(seed=3)
    gamma = w.gamma
    st = O.admm(s, B, lam_f, gamma, 4)
    nxt = O.admm(s, B, lam_f, gamma, 1, init=st)
    u = nxt.u
    for l in range(s.shape[0]):
        Au_v = O.forward(u[l], B)
        grad = s[l] + (O.adjoint(Au_v + st.b_v[l] - st.v[l], B) + (u[l] + st.b_w[l] - st.w[l])) / gamma
        assert np.max(np.abs(grad)) < 1e-12


def test_vw_updates_are_prox_points():
    # v^{i+1} minimises ||Lambda v||_1 + ||v - g_v||^2/(2 gamma) (subgradient test) and
    # w^{i+1} = P_C(g_w), b^{i+1} = g - y^{i+1}.
    s, B, lam_f, w = _problem(seed=4)
    st = O.admm(s, B, lam_f, w.gamma, 3)
    nxt = O.admm(s, B, lam_f, w.gamma, 1, init=st)
    thr = (w.gamma * lam_f)[:, None, None]
    for l in range(s.shape[0]):
        g_v = st.b_v[l] + O.forward(nxt.u[l], B)
        r = g_v - nxt.v[l]                        # must lie in gamma Lambda * subdiff|v|
        nz = nxt.v[l] != 0
        assert np.max(np.abs(np.where(nz, r - np.sign(nxt.v[l]) * thr, 0))) < 1e-12
        assert np.all(np.where(~nz, np.abs(r) <= thr + 1e-12, True))
        assert np.max(np.abs(nxt.b_v[l] - r)) < 1e-15
    g_w = st.b_w + nxt.u
    assert np.max(np.abs(nxt.w - O.project_simplex(g_w))) < 1e-15


def test_lambda_zero_gives_pointwise_argmin():
    s, B, lam_f, w = _problem(seed=5, lam=0.0)
    r1 = O.admm(s, B, lam_f * 0, w.gamma, 1)
    assert np.array_equal(r1.labels, np.argmin(s, axis=0))          # exact at iteration 1
    rK = O.admm(s, B, lam_f * 0, w.gamma, 60)
    srt = np.sort(s, axis=0)
    gap = srt[1] - srt[0]
    sel = gap > 0.05
    assert sel.mean() > 0.5
    assert np.array_equal(rK.labels[sel], np.argmin(s, axis=0)[sel])


def test_single_label_is_constant_one():
    s, B, lam_f, w = _problem(q=1, seed=6)
    r = O.admm(s, B, lam_f, w.gamma, 5)
    assert np.max(np.abs(r.w - 1.0)) < 1e-15 and np.all(r.labels == 0)


def test_scale_invariance_bitwise():
    # (s, Lambda, gamma) -> (2s, 2 Lambda, gamma/2) leaves every iterate unchanged exactly.
    s, B, lam_f, w = _problem(seed=7)
    a = O.admm(s, B, lam_f, w.gamma, 6)
    b = O.admm(2 * s, B, 2 * lam_f, w.gamma / 2, 6)
    for x, y in [(a.u, b.u), (a.v, b.v), (a.w, b.w), (a.b_v, b.b_v), (a.b_w, b.b_w)]:
        assert np.array_equal(x, y)


def test_label_permutation_and_transpose_and_shift():
    s, B, lam_f, w = _problem(seed=8, q=4)
    K = 8
    ref = O.admm(s, B, lam_f, w.gamma, K)
    perm = np.array([2, 0, 3, 1])
    rp = O.admm(s[perm], B, lam_f, w.gamma, K)
    assert np.max(np.abs(rp.w - ref.w[perm])) < 1e-13
    rt = O.admm(np.transpose(s, (0, 2, 1)).copy(), B, lam_f, w.gamma, K)
    assert np.max(np.abs(rt.w - np.transpose(ref.w, (0, 2, 1)))) < 1e-12
    rs = O.admm(np.roll(s, (3, -7), axis=(1, 2)), B, lam_f, w.gamma, K)
    assert np.max(np.abs(rs.w - np.roll(ref.w, (3, -7), axis=(1, 2)))) < 1e-12


def test_restart_equals_continuous_run():
    s, B, lam_f, w = _problem(seed=9)
    a = O.admm(s, B, lam_f, w.gamma, 7)
    b = O.admm(s, B, lam_f, w.gamma, 4)
    b = O.admm(s, B, lam_f, w.gamma, 3, init=b)
    assert np.array_equal(a.w, b.w) and np.array_equal(a.v, b.v) and np.array_equal(a.b_v, b.b_v)


def test_combined_residual_non_increasing_and_convergence():
    # For ADMM, ||y^{i+1}-y^i||^2 + ||b^{i+1}-b^i||^2 is non-increasing (He & Yuan's
    # non-ergodic analysis; the iteration is Douglas-Rachford, firmly non-expansive).
    s, B, lam_f, w = _problem(n=32, seed=10, lam=0.2)
    r = O.admm(s, B, lam_f, w.gamma, 150)
    c = r.r_combined
    assert np.all(np.diff(c) <= 1e-10 * c[:-1] + 1e-28)
    assert r.r_primal[-1] < 0.05 * r.r_primal[0] and r.r_dual[-1] < 0.05 * r.r_dual[0]
    # u - w -> 0 (primal feasibility of the split)
    assert np.max(np.abs(r.u - r.w)) < 0.05


def test_energy_beats_pointwise_labelling():
    s, B, lam_f, w = _problem(n=32, seed=11, lam=0.2)
    r = O.admm(s, B, lam_f, w.gamma, 150)
    onehot = (np.arange(s.shape[0])[:, None, None] == np.argmin(s, 0)[None]).astype(float)
    e_admm = O.energy(r.w, s, B, lam_f)
    assert e_admm < O.energy(onehot, s, B, lam_f)
    # the iterates' surrogate energy <w, s> + sum lambda |v| approaches the exact energy of w^K
    r30 = O.admm(s, B, lam_f, w.gamma, 30)
    gap30 = abs(r30.surrogate[-1] - O.energy(r30.w, s, B, lam_f))
    assert abs(r.surrogate[-1] - e_admm) < 0.5 * gap30


def test_fused_g_form_equals_literal_form():
    # The single-array recurrence used by the GPU library, written out here independently:
    #   g <- clip(g, +-gamma lambda) + S u,   v = g - clip(g),  b_v = clip(g),
    #   u = 1/2 [ S^T (g - 2 clip(g)) + (w - b_w) - gamma s ].
    s, B, lam_f, w = _problem(seed=12)
    gamma, K = w.gamma, 6
    ref = O.admm(s, B, lam_f, gamma, K)
    q, n, _ = s.shape
    thr = (gamma * lam_f)[:, None, None]
    g = np.zeros((q, B.shape[0], n, n))
    ww = np.zeros((q, n, n))
    bw = np.zeros((q, n, n))
    for _ in range(K):
        u = np.stack([0.5 * (O.adjoint(g[l] - 2 * np.clip(g[l], -thr, thr), B) + ww[l] - bw[l] - gamma * s[l])
                      for l in range(q)])
        for l in range(q):
            g[l] = np.clip(g[l], -thr, thr) + O.forward(u[l], B)
        gw = bw + u
        ww = O.project_simplex(gw)
        bw = gw - ww
    assert np.max(np.abs(ww - ref.w)) < 1e-12
    assert np.max(np.abs(g - np.clip(g, -thr[None], thr[None]) - ref.v)) < 1e-12


# ---- planted mistakes: each must be caught by one of the pins above -------------------

def _mutated(module, func_name, old, new):
    """Return a copy of `module.func_name` whose source has `old` replaced by `new`."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(getattr(module, func_name)))
    assert old in src
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), f"<mutant {func_name}>", "exec"), ns)
    return ns[func_name]


def test_planted_mistakes_are_caught():
    import oracle.filters as F
    import oracle.model as M
    import oracle.prox as P
    # (1) dropping the diagonal part of the glued seam filters breaks Theorem 2.2's identity
    ev = _mutated(F, "eval_filter", "return h + v + x", "return h + v")
    om = F.freq_index(32)
    B = np.stack([ev(kd, j, k, om[:, None], om[None, :], 16 / 32) for kd, j, k in F.filter_list(2)])
    assert np.max(np.abs(np.sum(B ** 2, 0) - 1)) > 0.1
    # (2) the integer grid (rho = 1) with J=2 at N=128 leaves the band (N/8, N/2] uncovered
    om = F.freq_index(128)
    Bl = np.stack([F.eval_filter(kd, j, k, om[:, None], om[None, :], 1.0) for kd, j, k in F.filter_list(2)])
    assert np.max(np.abs(np.sum(Bl ** 2, 0) - 1)) > 0.5
    # (3) a sign error on the data term of the u-update flips the lambda = 0 labelling
    s, B, lam_f, w = _problem(seed=5, lam=0.0)
    bad = _mutated(M, "admm", "- gamma * s[l])", "+ gamma * s[l])")
    assert not np.array_equal(bad(s, B, lam_f * 0, w.gamma, 1).labels, np.argmin(s, axis=0))
    # (4) a dropped 1/2 in the u-update violates the stationarity of the u-step
    bad = _mutated(M, "admm", "u[l] = 0.5 * (", "u[l] = 1.0 * (")
    st = M.admm(s, B, lam_f, w.gamma, 2)
    u = bad(s, B, lam_f, w.gamma, 1, init=st).u
    grad = s[0] + (M.adjoint(M.forward(u[0], B) + st.b_v[0] - st.v[0], B) + u[0] + st.b_w[0] - st.w[0]) / w.gamma
    assert np.max(np.abs(grad)) > 1e-3
    # (5) an off-by-one in the simplex threshold index disagrees with brute force
    bad_pc = _mutated(P, "project_simplex", "(rho - 1)[None]", "np.maximum(rho - 2, 0)[None]")
    g = np.random.default_rng(1).normal(size=(4, 200))
    assert np.max(np.abs(bad_pc(g) - P.project_simplex_bruteforce(g))) > 1e-3
