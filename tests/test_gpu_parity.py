"""GPU parity of the HIP library against the FP64 oracle, through the C ABI.

Tolerances (FP32 arithmetic on the GPU vs FP64 in the oracle):
* filter bank: max abs error <= 1e-6 (values in [0, 1], one FP32 rounding);
* transforms S and S^T: norm-relative error <= 1e-5 over the whole output;
* ADMM (FP32 storage): labels >= 99.9% identical, final energy within 1e-4 relative,
  relaxed labelling w^K within 1e-4 absolute (entries in [0, 1]).
"""
import numpy as np
import pytest

import oracle as O
from synth import make_c0, make_c1, make_c2, make_c4, make_small, random_data, random_image

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pkg():
    import paper_1112_1805_amd as pkg
    pkg.lib()
    return pkg


def dev_t(x, dtype=None):
    return torch.tensor(np.asarray(x), dtype=dtype or torch.float32, device="cuda:0")


def f32(x):
    """The float32 values the GPU sees, as float64 for the oracle."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


# ------------------------------------------------------------------ filter bank
@pytest.mark.parametrize("n,J", [(64, 1), (64, 2), (64, 3), (128, 2), (128, 3), (256, 4), (512, 3), (1024, 4)])
def test_filters_match_oracle(n, J):
    pkg = _pkg()
    plan = pkg.Plan(n, 1, 1, J)
    out = torch.empty((plan.eta, n, n // 2 + 1), dtype=torch.float32, device="cuda:0")
    plan.filters(out)
    torch.cuda.synchronize()
    ref = O.filter_bank(n, J)[:, :, : n // 2 + 1]
    assert np.max(np.abs(out.cpu().numpy() - ref)) < 1e-6


def test_filters_2048_sampled_columns():
    pkg = _pkg()
    n, J = 2048, 4
    plan = pkg.Plan(n, 1, 1, J)
    out = torch.empty((plan.eta, n, n // 2 + 1), dtype=torch.float32, device="cuda:0")
    plan.filters(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    om = O.freq_index(n)
    cols = [0, 1, 7, 128, 300, 511, 1023, 1024]
    from oracle.filters import eval_filter
    for f, (kind, j, k) in enumerate(O.filter_list(J)):
        ref = eval_filter(kind, j, k, om[:, None], om[None, cols], 4.0 ** J / n)
        # Nyquist bins are symmetrised: compare away from them, and check sum of squares there
        mask = np.ones_like(ref, dtype=bool)
        mask[n // 2, :] = False
        mask[:, np.array(cols) == n // 2] = False
        assert np.max(np.abs(got[f][:, cols][mask] - ref[mask])) < 1e-6
    assert np.max(np.abs(np.sum(got.astype(np.float64) ** 2, axis=0) - 1.0)) < 1e-6


# ------------------------------------------------------------------ transforms
TRANSFORM_CASES = [(64, 1, 1), (64, 3, 2), (128, 2, 3), (128, 3, 1), (256, 3, 2), (512, 3, 1), (1024, 4, 1)]


@pytest.mark.parametrize("n,J,count", TRANSFORM_CASES)
def test_forward_and_adjoint_match_oracle(n, J, count):
    pkg = _pkg()
    plan = pkg.Plan(n, 1, max(count, 2), J)
    ws = plan.new_workspace()
    f = random_image(n, seed=n + J, channels=count).astype(np.float32)
    c = torch.empty((count, plan.eta, n, n), dtype=torch.float32, device="cuda:0")
    plan.shearlet_forward(dev_t(f), c, ws)
    cd = random_data((count, plan.eta, n, n), seed=n * 3 + J).astype(np.float32)
    g = torch.empty((count, n, n), dtype=torch.float32, device="cuda:0")
    plan.shearlet_adjoint(dev_t(cd), g, ws)
    torch.cuda.synchronize()
    B = O.filter_bank(n, J)
    cg, gg = c.cpu().numpy(), g.cpu().numpy()
    for i in range(count):
        ref = O.forward(f32(f[i]), B)
        assert rel(cg[i], ref) < 1e-5
        # per filter, error relative to the image norm
        for jf in range(plan.eta):
            assert np.linalg.norm(cg[i, jf] - ref[jf]) < 1e-5 * np.linalg.norm(f[i])
        assert rel(gg[i], O.adjoint(f32(cd[i]), B)) < 1e-5


@pytest.mark.parametrize("n,J", [(1024, 4), (2048, 4)])
def test_parseval_and_reconstruction_full_size(n, J):
    # Properties that hold at any size (Theorem 2.2): ||S f|| = ||f||, S^T S f = f.
    pkg = _pkg()
    plan = pkg.Plan(n, 1, 1, J)
    ws = plan.new_workspace()
    f = dev_t(random_image(n, seed=5)[:1])
    c = torch.empty((1, plan.eta, n, n), dtype=torch.float32, device="cuda:0")
    plan.shearlet_forward(f, c, ws)
    r = torch.empty_like(f)
    plan.shearlet_adjoint(c, r, ws)
    torch.cuda.synchronize()
    nf = torch.linalg.vector_norm(f.double()).item()
    assert abs(torch.linalg.vector_norm(c.double()).item() / nf - 1) < 1e-5
    assert torch.linalg.vector_norm((r - f).double()).item() / nf < 1e-5
    # one filter image sampled against the oracle's filter j computed one by one
    fj = f[0].double().cpu().numpy()
    B = O.filter_bank(n, J)
    for jf in (0, 7, plan.eta - 1):
        ref = np.real(O.ifft2(B[jf] * O.fft2(fj)))
        assert np.linalg.norm(c[0, jf].double().cpu().numpy() - ref) < 1e-5 * np.linalg.norm(fj)


def test_transform_edge_cases():
    pkg = _pkg()
    n, J = 128, 2
    plan = pkg.Plan(n, 1, 2, J)
    ws = plan.new_workspace()
    c = torch.empty((1, plan.eta, n, n), dtype=torch.float32, device="cuda:0")
    # constant image: only the low-pass coefficient is nonzero, equal to the constant
    plan.shearlet_forward(torch.full((1, n, n), 0.7, device="cuda:0"), c, ws)
    torch.cuda.synchronize()
    assert torch.max(torch.abs(c[0, 0] - 0.7)).item() < 1e-6
    assert torch.max(torch.abs(c[0, 1:])).item() < 1e-6
    # zero image -> zero coefficients; impulse -> filters' impulse responses sum to delta
    plan.shearlet_forward(torch.zeros((1, n, n), device="cuda:0"), c, ws)
    torch.cuda.synchronize()
    assert torch.count_nonzero(c).item() == 0
    # count > q runs in groups of q: each image's coefficients equal its own transform
    f3 = dev_t(random_image(n, seed=21, channels=3))
    c3 = torch.empty((3, plan.eta, n, n), device="cuda:0")
    plan.shearlet_forward(f3, c3, ws)
    r3 = torch.empty_like(f3)
    plan.shearlet_adjoint(c3, r3, ws)
    torch.cuda.synchronize()
    for i in range(3):
        plan.shearlet_forward(f3[i:i + 1].contiguous(), c, ws)
        torch.cuda.synchronize()
        assert torch.equal(c[0], c3[i])
    assert torch.max(torch.abs(r3 - f3)).item() < 1e-5
    with pytest.raises(pkg.ShsError) as e:
        plan.shearlet_forward(torch.zeros((1, n, n), device="cuda:0"), c, ws[:1024])
    assert e.value.status == pkg.SHS_E_WORKSPACE


# ------------------------------------------------------------------ denoising S^T S_lambda S
DENOISE_CASES = [(64, 2, 2, 5), (128, 3, 3, 3), (96, 2, 2, 3), (160, 3, 4, 2), (256, 4, 1, 1), (512, 3, 2, 2)]


@pytest.mark.parametrize("n,J,q,count", DENOISE_CASES)
def test_denoise_matches_oracle(n, J, q, count):
    # count > q exercises the grouping; 96 and 160 the mixed-radix path
    pkg = _pkg()
    plan = pkg.Plan(n, 1, q, J)
    ws = plan.new_workspace()
    f = random_image(n, seed=7 * n + J, channels=count).astype(np.float32)
    rng = np.random.default_rng(n + count)
    lam_scale = np.float32([0.0] + list(rng.uniform(0.02, 0.3, size=J)))
    lam_filter = np.float32(rng.uniform(0.0, 0.3, size=plan.eta))
    B = O.filter_bank(n, J)
    for lam, lam_f in ((lam_scale, O.lambda_per_filter(f32(lam_scale), J)), (lam_filter, f32(lam_filter))):
        out = plan.shearlet_denoise(dev_t(f), lam, ws)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for i in range(count):
            ref = O.denoise(f32(f[i]), B, lam_f)
            assert np.linalg.norm(got[i] - ref) < 1e-5 * np.linalg.norm(f[i])


def test_denoise_full_size_and_edge_cases():
    pkg = _pkg()
    n, J = 1024, 4
    plan = pkg.Plan(n, 1, 2, J)
    ws = plan.new_workspace()
    f = random_image(n, seed=9, channels=2).astype(np.float32)
    fd = dev_t(f)
    # lambda = 0: the identity (Theorem 2.2)
    out0 = plan.shearlet_denoise(fd, np.zeros(J + 1, np.float32), ws)
    lam = np.float32([0.0, 0.05, 0.1, 0.2, 0.4])
    out = plan.shearlet_denoise(fd, lam, ws)
    # in place (d_out == d_f) gives the same bits
    fin = fd.clone()
    plan.shearlet_denoise(fin, lam, ws, out=fin)
    torch.cuda.synchronize()
    assert torch.linalg.vector_norm((out0 - fd).double()).item() < 1e-5 * torch.linalg.vector_norm(fd.double()).item()
    assert torch.equal(fin, out)
    ref = O.denoise(f32(f[1]), O.filter_bank(n, J), O.lambda_per_filter(f32(lam), J))
    assert np.linalg.norm(out[1].cpu().numpy() - ref) < 1e-5 * np.linalg.norm(f[1])
    # huge thresholds: zero output
    big = plan.shearlet_denoise(fd, np.full(J + 1, 1e30, np.float32), ws)
    torch.cuda.synchronize()
    assert torch.count_nonzero(big).item() == 0
    for bad in (np.float32([0.0, 0.1]), np.float32([0.0, -0.1, 0.1, 0.1, 0.1]),
                np.float32([0.0, np.nan, 0.1, 0.1, 0.1])):
        with pytest.raises(pkg.ShsError) as e:
            plan.shearlet_denoise(fd, bad, ws)
        assert e.value.status == pkg.SHS_E_INVALID


# ------------------------------------------------------------------ data term
@pytest.mark.parametrize("channels,q", [(1, 3), (3, 5), (3, 8), (4, 2)])
def test_datacost(channels, q):
    pkg = _pkg()
    n = 128
    w = make_small(n, q, 2, channels=channels, seed=channels * 10 + q)
    plan = pkg.Plan(n, channels, q, 2)
    s = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
    plan.datacost(dev_t(w.img), w.codebook, s)
    torch.cuda.synchronize()
    ref = O.datacost(f32(w.img), f32(w.codebook))
    assert np.max(np.abs(s.cpu().numpy() - ref)) < 1e-5 * max(1.0, ref.max())
    s1 = torch.empty_like(s)
    plan.datacost(dev_t(w.img), w.codebook, s1, p=1.0)
    torch.cuda.synchronize()
    assert np.max(np.abs(s1.cpu().numpy() - O.datacost(f32(w.img), f32(w.codebook), p=1))) < 1e-5


# ------------------------------------------------------------------ ADMM solve
def run_gpu(w, iters=None, store="f32", hist=True, s=None, lam=None, gamma=None, plan=None, ws=None,
            resume=False, want_stats=True):
    pkg = _pkg()
    iters = w.iters if iters is None else iters
    n, q, C = w.n, w.q, w.channels
    plan = plan or pkg.Plan(n, C, q, w.J, store)
    ws = plan.new_workspace() if ws is None else ws
    if s is None:
        s = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
        plan.datacost(dev_t(w.img), w.codebook, s)
    u = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
    labels = torch.empty((n, n), dtype=torch.int32, device="cuda:0")
    h = torch.zeros((iters, 4), dtype=torch.float64, device="cuda:0") if hist and iters > 0 else None
    st = plan.solve(s, ws, w.lam if lam is None else lam, w.gamma if gamma is None else gamma, iters,
                    u=u, labels=labels, hist=h, resume=resume, want_stats=want_stats)
    torch.cuda.synchronize()
    return dict(u=u.cpu().numpy(), labels=labels.cpu().numpy(), stats=st,
                hist=None if h is None else h.cpu().numpy(), s=s, plan=plan, ws=ws)


def run_oracle(w, iters=None, s=None):
    iters = w.iters if iters is None else iters
    s = O.datacost(f32(w.img), f32(w.codebook)) if s is None else s
    B = O.filter_bank(w.n, w.J)
    lam_f = O.lambda_per_filter(w.lam, w.J)
    r = O.admm(s, B, lam_f, w.gamma, iters)
    return r, s, B, lam_f


def compare_solution(g, r, s, B, lam_f, atol_u=1e-4, label_frac=0.999, e_rel=1e-4):
    du = np.max(np.abs(g["u"] - r.w))
    agree = np.mean(g["labels"] == r.labels)
    e_ref = O.energy(r.w, s, B, lam_f)
    de = abs(g["stats"]["energy"] - e_ref) / abs(e_ref)
    print(f"max|u-u_ref|={du:.3e} labels={agree:.6f} energy rel={de:.3e}")
    assert agree >= label_frac
    assert de <= e_rel
    assert du <= atol_u
    return du, agree, de


@pytest.fixture(scope="module")
def c0_pair():
    w = make_c0()
    r, s, B, lam_f = run_oracle(w)
    g = run_gpu(w)
    return w, g, r, s, B, lam_f


def test_c0_full_run_parity(c0_pair):
    w, g, r, s, B, lam_f = c0_pair
    compare_solution(g, r, s, B, lam_f)
    assert g["stats"]["iters_done"] == w.iters
    # residual histories follow the oracle's
    h = g["hist"]
    for col, ref in [(0, r.r_primal), (1, r.r_dual), (2, r.r_combined), (3, r.surrogate)]:
        err = np.abs(h[:, col] - ref) / np.maximum(np.abs(ref), 1e-12)
        assert np.median(err) < 1e-3, (col, np.median(err))
        assert err[:50].max() < 1e-2, (col, err[:50].max())
    # He-Yuan: the combined residual is non-increasing (up to FP32 noise)
    c = h[:, 2]
    assert np.all(np.diff(c) <= 1e-3 * c[:-1] + 1e-12)


def test_c0_outputs_valid(c0_pair):
    w, g, r, s, B, lam_f = c0_pair
    u = g["u"]
    assert np.all(u >= 0) and np.max(np.abs(u.sum(0) - 1)) < 1e-5     # u* in C
    assert np.array_equal(g["labels"], np.argmax(u, axis=0))           # argmax, first index


@pytest.mark.parametrize("n,q,J,C,iters", [(64, 1, 1, 1, 5), (64, 2, 3, 1, 15), (64, 8, 2, 3, 10),
                                           (128, 5, 3, 3, 12), (256, 4, 2, 1, 8), (256, 6, 4, 1, 6)])
def test_small_solves_elementwise(n, q, J, C, iters):
    w = make_small(n, q, J, channels=C, seed=n + q + J, lam=0.15, gamma=1.0, iters=iters)
    r, s, B, lam_f = run_oracle(w)
    g = run_gpu(w)
    du = np.max(np.abs(g["u"] - r.w))
    assert du < 2e-5, du
    assert np.mean(g["labels"] == r.labels) >= 0.999
    if q == 1:
        assert np.all(g["u"] == 1.0) and np.all(g["labels"] == 0)


def test_c1_prefix_parity():
    w = make_c1()
    K = 12
    r, s, B, lam_f = run_oracle(w, iters=K)
    g = run_gpu(w, iters=K)
    compare_solution(g, r, s, B, lam_f, atol_u=2e-5)
    h = g["hist"]
    assert np.max(np.abs(h[:, 2] - r.r_combined) / r.r_combined) < 1e-3


@pytest.mark.parametrize("store,atol_u,e_rel", [("f32", 2e-5, 1e-5), ("f16", 5e-3, 1e-3), ("bf16", 3e-2, 1e-2)])
def test_c2_full_size_prefix(store, atol_u, e_rel):
    # Full 1024^2 RGB, q=5, J=4 (61 filters) in the launch configuration of the benchmark;
    # the oracle runs a 2-iteration prefix.
    w = make_c2()
    K = 2
    key = "_c2_oracle"
    cache = test_c2_full_size_prefix.__dict__
    if key not in cache:
        cache[key] = run_oracle(w, iters=K)
    r, s, B, lam_f = cache[key]
    g = run_gpu(w, iters=K, store=store)
    du = np.max(np.abs(g["u"] - r.w))
    e_ref = O.energy(r.w, s, B, lam_f)
    de = abs(g["stats"]["energy"] - e_ref) / abs(e_ref)
    print(store, du, de)
    assert du < atol_u and de < e_rel
    assert np.mean(g["labels"] == r.labels) >= 0.999


def test_c4_full_size_properties():
    # 2048^2 gray, q=8, J=4 (61 filters), BF16 state: the benchmark's C4 launch configuration.
    # The oracle's full-size coefficient arrays do not fit a test, so this checks what is fixed
    # at any size: the data term elementwise; after one iteration from zero, u^1 = -gamma s / 2
    # and w^1 = P_C(u^1) exactly (Section 3 updates with v = w = b = 0); later iterates stay in
    # C with argmax labels and a non-increasing combined residual (He & Yuan).
    w = make_c4()
    g1 = run_gpu(w, iters=1, store="bf16")
    s = g1["s"].double().cpu().numpy()
    s_ref = O.datacost(f32(w.img), f32(w.codebook))
    assert np.max(np.abs(s - s_ref)) < 1e-6 * max(1.0, np.max(np.abs(s_ref)))
    w1 = O.project_simplex(-0.5 * w.gamma * s)
    assert np.max(np.abs(g1["u"] - w1)) < 1e-5
    gap = np.sort(s, axis=0)
    clear = gap[1] - gap[0] > 1e-5
    assert np.array_equal(g1["labels"][clear], np.argmin(s, axis=0)[clear])
    gk = run_gpu(w, iters=5, store="bf16", s=g1["s"], plan=g1["plan"], ws=g1["ws"])
    h = gk["hist"]
    assert np.all(np.isfinite(h))
    c = h[:, 2]
    assert np.all(np.diff(c) <= 1e-2 * c[:-1] + 1e-12), c     # BF16-stored state: 1e-2 slack
    u = gk["u"]
    assert np.all(u >= 0) and np.max(np.abs(u.sum(0) - 1)) < 1e-5
    assert np.array_equal(gk["labels"], np.argmax(u, axis=0))
    assert np.isfinite(gk["stats"]["energy"]) and gk["stats"]["iters_done"] == 5


# ------------------------------------------------------------------ primal-dual solver
def run_gpu_pd(w, iters, tau, sigma, store="f32", lam=None, s=None):
    pkg = _pkg()
    n, q = w.n, w.q
    plan = pkg.Plan(n, w.channels, q, w.J, store)
    ws = plan.new_workspace()
    if s is None:
        s = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
        plan.datacost(dev_t(w.img), w.codebook, s)
    u = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
    labels = torch.empty((n, n), dtype=torch.int32, device="cuda:0")
    h = torch.zeros((iters, 4), dtype=torch.float64, device="cuda:0")
    st = plan.solve_pd(s, ws, w.lam if lam is None else lam, tau, sigma, iters, u=u, labels=labels, hist=h)
    torch.cuda.synchronize()
    return dict(u=u.cpu().numpy(), labels=labels.cpu().numpy(), stats=st, hist=h.cpu().numpy(), s=s,
                plan=plan, ws=ws)


PD_CASES = [(64, 3, 2, 1, 30, 0.9, 0.9), (64, 1, 1, 1, 5, 1.0, 1.0), (128, 5, 3, 3, 20, 2.0, 0.5),
            (96, 4, 2, 1, 20, 0.9, 0.9), (160, 2, 3, 1, 15, 1.0, 1.0), (256, 8, 4, 1, 10, 0.5, 2.0)]


@pytest.mark.parametrize("n,q,J,C,iters,tau,sigma", PD_CASES)
def test_primal_dual_matches_oracle(n, q, J, C, iters, tau, sigma):
    w = make_small(n, q, J, channels=C, seed=3 * n + q, lam=0.15, iters=iters)
    s = O.datacost(f32(w.img), f32(w.codebook))
    B = O.filter_bank(n, J)
    lam_f = O.lambda_per_filter(w.lam, J)
    r = O.primal_dual(s, B, lam_f, tau, sigma, iters)
    g = run_gpu_pd(w, iters, tau, sigma)
    assert np.max(np.abs(g["u"] - r.u)) < 5e-5
    assert np.mean(g["labels"] == r.labels) >= 0.999
    # per-iteration history: ||du||, ||dy|| (relative to the sequence's size), surrogate
    assert np.max(np.abs(g["hist"][:, 0] - r.du)) < 1e-4 * np.max(r.du)
    assert np.max(np.abs(g["hist"][:, 1] - r.dy)) < 1e-4 * max(np.max(r.dy), 1e-30)
    assert np.max(np.abs(g["hist"][:, 3] - r.surrogate) / np.abs(r.surrogate)) < 1e-5
    e_ref = O.energy(r.u, s, B, lam_f)
    assert abs(g["stats"]["energy"] - e_ref) < 1e-4 * abs(e_ref)
    if q == 1:
        assert np.all(g["u"] == 1.0) and np.all(g["labels"] == 0)


@pytest.mark.parametrize("store,atol_u,e_rel", [("f32", 2e-5, 1e-5), ("f16", 5e-3, 1e-3)])
def test_primal_dual_c2_full_size_prefix(store, atol_u, e_rel):
    # 1024^2 RGB, q=5, J=4 in the benchmark's launch configuration; 2 oracle iterations
    w = make_c2()
    K, tau, sigma = 2, 2.0, 0.5
    key = "_pd_c2_oracle"
    cache = test_primal_dual_c2_full_size_prefix.__dict__
    if key not in cache:
        s = O.datacost(f32(w.img), f32(w.codebook))
        B = O.filter_bank(w.n, w.J)
        lam_f = O.lambda_per_filter(w.lam, w.J)
        cache[key] = (O.primal_dual(s, B, lam_f, tau, sigma, K), s, B, lam_f)
    r, s, B, lam_f = cache[key]
    g = run_gpu_pd(w, K, tau, sigma, store=store)
    assert np.max(np.abs(g["u"] - r.u)) < atol_u
    e_ref = O.energy(r.u, s, B, lam_f)
    assert abs(g["stats"]["energy"] - e_ref) < e_rel * abs(e_ref)
    assert np.mean(g["labels"] == r.labels) >= 0.999


def test_primal_dual_and_admm_reach_the_same_minimum():
    # both solvers minimise the same convex functional: their energies meet (GPU only)
    w = make_small(64, 3, 2, seed=8, lam=0.1, iters=1)
    pd = run_gpu_pd(w, 3000, 0.9, 0.9)
    ad = run_gpu(w, iters=3000, hist=False)
    e_pd, e_ad = pd["stats"]["energy"], ad["stats"]["energy"]
    assert abs(e_pd - e_ad) < 1e-4 * abs(e_ad)
    assert np.mean(pd["labels"] == ad["labels"]) > 0.99


def test_primal_dual_lambda_zero_and_errors():
    pkg = _pkg()
    w = make_small(128, 4, 2, seed=3, lam=0.0, iters=1)
    g = run_gpu_pd(w, 2, 1e4, 1e-4)
    s = g["s"].cpu().numpy()
    assert np.array_equal(g["labels"], np.argmin(s, axis=0))
    plan, ws, sd = g["plan"], g["ws"], g["s"]
    for tau, sigma, lam in ((1.0, 1.5, w.lam), (0.0, 1.0, w.lam), (1.0, float("nan"), w.lam),
                            (1.0, 1.0, [0.1, 0.2]), (1.0, 1.0, [0.0, -0.1, 0.1])):
        with pytest.raises(pkg.ShsError) as e:
            plan.solve_pd(sd, ws, lam, tau, sigma, 2)
        assert e.value.status == pkg.SHS_E_INVALID


# ------------------------------------------------------------------ TV comparison model
def run_gpu_tv(w, iters, lam, gamma=1.0, store="f32"):
    pkg = _pkg()
    n, q = w.n, w.q
    plan = pkg.Plan(n, w.channels, q, w.J, store)
    ws = plan.new_workspace()
    s = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
    plan.datacost(dev_t(w.img), w.codebook, s)
    u = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
    labels = torch.empty((n, n), dtype=torch.int32, device="cuda:0")
    h = torch.zeros((max(iters, 1), 4), dtype=torch.float64, device="cuda:0")
    st = plan.solve_tv(s, ws, lam, gamma, iters, u=u, labels=labels, hist=h[:iters] if iters else None)
    torch.cuda.synchronize()
    return dict(u=u.cpu().numpy(), labels=labels.cpu().numpy(), stats=st, hist=h.cpu().numpy()[:iters], s=s,
                plan=plan, ws=ws)


TV_CASES = [(64, 3, 1, 20, 0.2, 1.0), (128, 5, 3, 15, 0.1, 0.5), (96, 4, 1, 15, 0.2, 1.0),
            (160, 2, 1, 10, 0.3, 2.0), (256, 8, 1, 8, 0.05, 1.0), (64, 1, 1, 5, 0.2, 1.0)]


@pytest.mark.parametrize("n,q,C,iters,lam,gamma", TV_CASES)
def test_tv_matches_oracle(n, q, C, iters, lam, gamma):
    w = make_small(n, q, 1, channels=C, seed=5 * n + q, iters=iters)
    s = O.datacost(f32(w.img), f32(w.codebook))
    r = O.tv_admm(s, lam, gamma, iters)
    g = run_gpu_tv(w, iters, lam, gamma)
    assert np.max(np.abs(g["u"] - r.w)) < 5e-5
    assert np.mean(g["labels"] == r.labels) >= 0.999
    assert np.max(np.abs(g["hist"][:, 0] - r.r_primal)) < 1e-4 * np.max(r.r_primal)
    assert np.max(np.abs(g["hist"][:, 1] - r.r_dual)) < 1e-4 * np.max(r.r_dual)
    assert np.max(np.abs(g["hist"][:, 3] - r.surrogate) / np.abs(r.surrogate)) < 1e-5
    e_ref = O.tv_energy(r.w, s, lam)
    assert abs(g["stats"]["energy"] - e_ref) < 1e-5 * abs(e_ref)
    if q == 1:
        assert np.all(g["u"] == 1.0)


@pytest.mark.parametrize("store,atol_u,e_rel", [("f32", 2e-5, 1e-5), ("f16", 5e-3, 1e-3), ("bf16", 3e-2, 1e-2)])
def test_tv_c2_full_size_prefix(store, atol_u, e_rel):
    w = make_c2()
    K, lam, gamma = 3, 0.05, 1.0
    key = "_tv_c2_oracle"
    cache = test_tv_c2_full_size_prefix.__dict__
    if key not in cache:
        s = O.datacost(f32(w.img), f32(w.codebook))
        cache[key] = (O.tv_admm(s, lam, gamma, K), s)
    r, s = cache[key]
    g = run_gpu_tv(w, K, lam, gamma, store=store)
    assert np.max(np.abs(g["u"] - r.w)) < atol_u
    e_ref = O.tv_energy(r.w, s, lam)
    assert abs(g["stats"]["energy"] - e_ref) < e_rel * abs(e_ref)
    assert np.mean(g["labels"] == r.labels) >= 0.999


def test_tv_errors_and_zero_iterations():
    pkg = _pkg()
    w = make_small(64, 3, 1, seed=2, iters=1)
    g = run_gpu_tv(w, 0, 0.1)
    assert np.all(g["u"] == 0.0)
    plan, ws, s = g["plan"], g["ws"], g["s"]
    for lam, gamma in (([0.1, 0.2], 1.0), ([-0.1], 1.0), ([float("inf")], 1.0), ([0.1], 0.0)):
        prm_lam = lam if len(lam) != 1 else lam[0]
        with pytest.raises(pkg.ShsError) as e:
            if len(lam) == 1:
                plan.solve_tv(s, ws, prm_lam, gamma, 2)
            else:
                prm, keep = pkg._params(lam, gamma, 2)
                pkg._check(pkg.lib().shs_solve_tv(plan.handle, pkg.ctypes.byref(prm), pkg._ptr(s), pkg._ptr(ws),
                                                  ws.numel(), None, None, None, None, pkg._stream(None)), "tv")
        assert e.value.status == pkg.SHS_E_INVALID


# ------------------------------------------------------------------ NL (graph) model
def run_gpu_nl(w, iters, lam, store="f32", J=2, m=5, graph=None, tau=None, sigma=None):
    pkg = _pkg()
    n, q = w.n, w.q
    nbr, rev, md = graph if graph is not None else pkg.nl_graph(np.float32(w.img), 5, 15, 2.0, m)
    tau = tau if tau is not None else 1.0 / np.sqrt(4.0 * md)
    sigma = sigma if sigma is not None else 1.0 / np.sqrt(4.0 * md)
    plan = pkg.Plan(n, w.channels, q, J, store)
    ws = plan.new_workspace()
    s = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
    plan.datacost(dev_t(w.img), w.codebook, s)
    u = torch.empty((q, n, n), dtype=torch.float32, device="cuda:0")
    labels = torch.empty((n, n), dtype=torch.int32, device="cuda:0")
    h = torch.zeros((iters, 4), dtype=torch.float64, device="cuda:0")
    st = plan.solve_nl(s, dev_t(nbr, torch.int32), dev_t(rev, torch.int32), ws, lam, tau, sigma, iters, md,
                       u=u, labels=labels, hist=h)
    torch.cuda.synchronize()
    return dict(u=u.cpu().numpy(), labels=labels.cpu().numpy(), stats=st, hist=h.cpu().numpy(), s=s,
                plan=plan, ws=ws, nbr=nbr, rev=rev, md=md, tau=tau, sigma=sigma)


NL_CASES = [(64, 3, 1, 20, 0.1), (96, 5, 3, 15, 0.05), (72, 2, 1, 10, 0.2), (128, 8, 1, 8, 0.05), (64, 1, 1, 5, 0.1)]


@pytest.mark.parametrize("n,q,C,iters,lam", NL_CASES)
def test_nl_matches_oracle(n, q, C, iters, lam):
    w = make_small(n, q, 2, channels=C, seed=7 * n + q, iters=iters)
    g = run_gpu_nl(w, iters, lam)
    s = O.datacost(f32(w.img), f32(w.codebook))
    nbr = g["nbr"].astype(np.int64)
    r = O.nl_primal_dual(s, nbr, lam, g["tau"], g["sigma"], iters)
    assert np.max(np.abs(g["u"] - r.u)) < 5e-5
    assert np.mean(g["labels"] == r.labels) >= 0.999
    assert np.max(np.abs(g["hist"][:, 0] - r.du)) < 1e-4 * np.max(r.du)
    # floor: with q = 1 the dual changes are rounding noise on both sides (the oracle's
    # FP64 projection leaves u = 1 up to ~1e-16, so its graph differences give |dy| ~ 4e-15
    # where the GPU's are exactly 0); below 1e-9 the relative bound becomes absolute (1e-13)
    assert np.max(np.abs(g["hist"][:, 1] - r.dy)) < 1e-4 * max(np.max(r.dy), 1e-9)
    assert np.max(np.abs(g["hist"][:, 3] - r.surrogate) / np.abs(r.surrogate)) < 1e-5
    e_ref = O.nl_energy(r.u, s, nbr, lam)
    assert abs(g["stats"]["energy"] - e_ref) < 1e-5 * abs(e_ref)
    if q == 1:
        assert np.all(g["u"] == 1.0)


@pytest.mark.parametrize("store,atol_u", [("f32", 2e-5), ("f16", 5e-3)])
def test_nl_c2_full_size_prefix(store, atol_u):
    # 1024^2 RGB, q=5: the library's graph (its parity with the oracle's construction is a
    # CPU test) and 2 oracle primal-dual iterations on it
    w = make_c2()
    key = "_nl_c2"
    cache = test_nl_c2_full_size_prefix.__dict__
    pkg = _pkg()
    if key not in cache:
        graph = pkg.nl_graph(np.float32(w.img), 5, 15, 2.0, 5)
        s = O.datacost(f32(w.img), f32(w.codebook))
        t = 1.0 / np.sqrt(4.0 * graph[2])
        cache[key] = (graph, O.nl_primal_dual(s, graph[0].astype(np.int64), 0.02, t, t, 2), s)
    graph, r, s = cache[key]
    g = run_gpu_nl(w, 2, 0.02, store=store, J=4, graph=graph)
    assert np.max(np.abs(g["u"] - r.u)) < atol_u
    assert np.mean(g["labels"] == r.labels) >= 0.999


def test_nl_errors():
    pkg = _pkg()
    w = make_small(64, 3, 2, seed=9, iters=1)
    g = run_gpu_nl(w, 1, 0.1)
    plan, ws, s, nbr, rev, md = g["plan"], g["ws"], g["s"], g["nbr"], g["rev"], g["md"]
    dn, dr = dev_t(nbr, torch.int32), dev_t(rev, torch.int32)
    with pytest.raises(pkg.ShsError) as e:                 # steps too large for ||D||^2 <= 4 max degree
        plan.solve_nl(s, dn, dr, ws, 0.1, 1.0, 1.0, 2, md)
    assert e.value.status == pkg.SHS_E_INVALID
    with pytest.raises(pkg.ShsError) as e:                 # negative weight
        plan.solve_nl(s, dn, dr, ws, -0.1, 0.1, 0.1, 2, md)
    assert e.value.status == pkg.SHS_E_INVALID
    small = pkg.Plan(64, 1, 3, 1)                          # eta = 5 < 2m = 10 blocks
    with pytest.raises(pkg.ShsError) as e:
        small.solve_nl(s, dn, dr, small.new_workspace(), 0.1, 0.1, 0.1, 2, md)
    assert e.value.status == pkg.SHS_E_UNSUPPORTED


def test_lambda_zero_argmin_exact():
    w = make_small(128, 4, 2, seed=3, lam=0.0, iters=1)
    g = run_gpu(w, iters=1)
    s32 = g["s"].cpu().numpy()
    assert np.array_equal(g["labels"], np.argmin(s32, axis=0))


# ------------------------------------------------------------------ invariances
def test_scale_invariance_bitwise():
    w = make_small(128, 3, 2, seed=21, lam=0.1, iters=15)
    a = run_gpu(w)
    b = run_gpu(w, s=a["s"] * 2, lam=w.lam * 2, gamma=w.gamma / 2)
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["labels"], b["labels"])


def test_label_permutation_transpose_shift():
    w = make_small(128, 4, 2, seed=22, lam=0.1, iters=10)
    a = run_gpu(w)
    perm = [2, 0, 3, 1]
    b = run_gpu(w, s=a["s"][perm].contiguous())
    assert np.max(np.abs(b["u"] - a["u"][perm])) < 2e-6
    c = run_gpu(w, s=a["s"].transpose(1, 2).contiguous())
    assert np.max(np.abs(c["u"] - np.transpose(a["u"], (0, 2, 1)))) < 2e-6
    d = run_gpu(w, s=torch.roll(a["s"], (5, -9), dims=(1, 2)).contiguous())
    assert np.max(np.abs(d["u"] - np.roll(a["u"], (5, -9), axis=(1, 2)))) < 2e-6


@pytest.mark.parametrize("store,n", [("f32", 128), ("bf16", 128), ("f16", 512), ("f32", 1024)])
def test_resume_bitwise(store, n):
    # n = 512 and 1024 run the two-rows-per-wavefront row pass (its restart primes the
    # adjoint input from the stored state)
    w = make_small(n, 3, 3, seed=23, lam=0.1, iters=14)
    full = run_gpu(w, store=store, hist=False)
    part = run_gpu(w, iters=9, store=store, hist=False)
    # checkpoint: copy the state prefix out, scribble, copy back, resume
    nb = part["plan"].state_bytes()
    saved = part["ws"][:nb].clone()
    part["ws"][:nb].zero_()
    part["ws"][:nb].copy_(saved)
    rest = run_gpu(w, iters=5, store=store, hist=False, s=part["s"], plan=part["plan"], ws=part["ws"],
                   resume=True)
    assert np.array_equal(full["u"], rest["u"])


# ------------------------------------------------------------------ errors and stopping
def test_error_paths():
    pkg = _pkg()
    w = make_small(64, 2, 1, seed=1, iters=3)
    plan = pkg.Plan(64, 1, 2, 1)
    ws = plan.new_workspace()
    s = torch.zeros((2, 64, 64), device="cuda:0")
    with pytest.raises(pkg.ShsError) as e:
        plan.solve(s, ws[:100], w.lam, 1.0, 3)
    assert e.value.status == pkg.SHS_E_WORKSPACE
    with pytest.raises(pkg.ShsError) as e:
        plan.solve(s, ws, [0.1, 0.2, 0.3], 1.0, 3)           # lambda_len neither J+1 nor eta
    assert e.value.status == pkg.SHS_E_INVALID
    with pytest.raises(pkg.ShsError):
        plan.solve(s, ws, w.lam, 0.0, 3)                    # gamma <= 0
    with pytest.raises(pkg.ShsError):
        plan.solve(s, ws, [0.0, -1.0], 1.0, 3)              # negative weight
    # NaN data term -> SHS_E_NUMERIC at the checked iteration
    with pytest.raises(pkg.ShsError) as e:
        plan.solve(torch.full((2, 64, 64), float("nan"), device="cuda:0"), ws, w.lam, 1.0, 3)
    assert e.value.status == pkg.SHS_E_NUMERIC


def test_f16_state_overflow_is_reported():
    # FP16 state holds |g| < 65504; a data term far above that range (an unscaled 8-bit
    # image with gamma = 1) overflows the stored coefficients, and the solve reports it
    # even when no statistics are requested.
    pkg = _pkg()
    plan = pkg.Plan(64, 1, 3, 2, "f16")
    ws = plan.new_workspace()
    s = torch.full((3, 64, 64), 4.0e5, device="cuda:0")
    s[1, :32] = 0.0
    with pytest.raises(pkg.ShsError) as e:
        plan.solve(s, ws, [0.0, 0.1, 0.1], 1.0, 3, want_stats=False)
    assert e.value.status == pkg.SHS_E_NUMERIC
    # the same problem scaled into range solves
    plan.solve(s / 1e5, ws, [0.0, 0.1, 0.1], 1.0, 3, want_stats=False)


def test_zero_iterations_and_tolerance_stop():
    w = make_small(64, 3, 2, seed=4, lam=0.1, iters=0)
    g = run_gpu(w, iters=0)
    assert np.all(g["u"] == 0) and g["stats"]["iters_done"] == 0
    pkg = _pkg()
    w = make_small(64, 3, 2, seed=4, lam=0.1, iters=50)
    plan = pkg.Plan(64, 1, 3, 2)
    ws = plan.new_workspace()
    s = torch.empty((3, 64, 64), device="cuda:0")
    plan.datacost(dev_t(w.img), w.codebook, s)
    st = plan.solve(s, ws, w.lam, 1.0, 50, tol=1e-2, check_every=5)
    assert st["iters_done"] < 50 and st["iters_done"] % 5 == 0
    assert np.sqrt(st["r_combined"]) <= 1e-2 * np.sqrt(3 * 64 * 64)


def test_profile_times_only_selected_classes():
    # event timing of chosen kernel classes does not change results; only those classes report
    pkg = _pkg()
    w = make_small(64, 3, 2, seed=5, lam=0.1, iters=6)
    plan = pkg.Plan(64, 1, 3, 2)
    ws = plan.new_workspace()
    s = torch.empty((3, 64, 64), device="cuda:0")
    plan.datacost(dev_t(w.img), w.codebook, s)
    u0 = torch.empty_like(s)
    plan.solve(s, ws, w.lam, 1.0, 6, u=u0)
    pkg.shs_profile_begin(["row_solve", "pixel"])
    u1 = torch.empty_like(s)
    plan.solve(s, ws, w.lam, 1.0, 6, u=u1)
    torch.cuda.synchronize()
    prof = pkg.shs_profile_end()
    assert set(prof) == {"row_solve", "pixel"}
    assert prof["row_solve"][0] >= 5 and prof["pixel"][0] >= 5
    assert all(ms > 0 for _, ms in prof.values())
    assert torch.equal(u0, u1)
    pkg.shs_profile_begin()
    plan.solve(s, ws, w.lam, 1.0, 6, u=u1)
    torch.cuda.synchronize()
    prof = pkg.shs_profile_end()
    assert {"row_solve", "pixel", "col_syn", "col_ana"} <= set(prof)


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_graph_replayed_iterations_equal_eager(store):
    # Steady-state iterations are replayed from captured graphs when no kernel timing is on;
    # with timing on every launch is eager.  Same bits either way, also for the history rows
    # (written through the device row counter), on a cache hit, after a re-capture for other
    # parameters, and with eager library work between replays.
    pkg = _pkg()
    w = make_small(96, 3, 2, seed=17, lam=0.1, iters=29)
    plan = pkg.Plan(96, 1, 3, 2, store)
    ws = plan.new_workspace()
    s = torch.empty((3, 96, 96), device="cuda:0")
    plan.datacost(dev_t(w.img), w.codebook, s)

    def run(lam, timed):
        u = torch.empty_like(s)
        lab = torch.empty((96, 96), dtype=torch.int32, device="cuda:0")
        h = torch.zeros((w.iters, 4), dtype=torch.float64, device="cuda:0")
        if timed:
            pkg.shs_profile_begin(["pixel"])
        st = plan.solve(s, ws, lam, 1.0, w.iters, u=u, labels=lab, hist=h)
        torch.cuda.synchronize()
        if timed:
            pkg.shs_profile_end()
        return u.cpu().numpy(), lab.cpu().numpy(), h.cpu().numpy(), st

    ws2 = plan.new_workspace()
    coef = torch.empty((1, plan.eta, 96, 96), device="cuda:0")
    for lam in (w.lam, w.lam * 1.5, w.lam):
        ref = run(lam, True)
        for rep in range(2):
            got = run(lam, False)
            plan.shearlet_forward(s[:1].contiguous(), coef, ws2)   # eager work between replays
            for a, b in zip(ref[:3], got[:3]):
                assert np.array_equal(a, b), (lam, rep)
            assert ref[3] == got[3]
    assert np.all(ref[2][:, 2] > 0)


def test_energy_entry_point():
    pkg = _pkg()
    w = make_small(128, 3, 2, seed=8)
    plan = pkg.Plan(128, 1, 3, 2)
    ws = plan.new_workspace()
    s = torch.empty((3, 128, 128), device="cuda:0")
    plan.datacost(dev_t(w.img), w.codebook, s)
    u = np.random.default_rng(0).uniform(size=(3, 128, 128)).astype(np.float32)
    e = plan.energy(s, dev_t(u), ws, w.lam)
    ref = O.energy(f32(u), f32(s.cpu().numpy()), O.filter_bank(128, 2), O.lambda_per_filter(w.lam, 2))
    assert abs(e - ref) / abs(ref) < 1e-6


# ------------------------------------------------------------------ mixed-radix sizes
# Image sides 32 * m (the sizes of a mixed batch) run the generic mixed-radix path.
MIXED = [(96, 2, 1), (160, 3, 2), (224, 3, 1), (352, 3, 1), (480, 3, 2), (608, 3, 1), (736, 3, 1), (768, 3, 1)]


@pytest.mark.parametrize("n,J,count", MIXED)
def test_mixed_radix_transforms(n, J, count):
    pkg = _pkg()
    plan = pkg.Plan(n, 1, max(count, 2), J)
    ws = plan.new_workspace()
    f = random_image(n, seed=n + 7, channels=count).astype(np.float32)
    c = torch.empty((count, plan.eta, n, n), dtype=torch.float32, device="cuda:0")
    plan.shearlet_forward(dev_t(f), c, ws)
    cd = random_data((count, plan.eta, n, n), seed=n * 5).astype(np.float32)
    g = torch.empty((count, n, n), dtype=torch.float32, device="cuda:0")
    plan.shearlet_adjoint(dev_t(cd), g, ws)
    psi = torch.empty((plan.eta, n, n // 2 + 1), dtype=torch.float32, device="cuda:0")
    plan.filters(psi)
    torch.cuda.synchronize()
    B = O.filter_bank(n, J)
    assert np.max(np.abs(psi.cpu().numpy() - B[:, :, : n // 2 + 1])) < 1e-6
    cg, gg = c.cpu().numpy(), g.cpu().numpy()
    for i in range(count):
        assert rel(cg[i], O.forward(f32(f[i]), B)) < 1e-5
        assert rel(gg[i], O.adjoint(f32(cd[i]), B)) < 1e-5


@pytest.mark.parametrize("n,q,J,C,iters", [(96, 3, 2, 1, 20), (160, 6, 3, 1, 12), (352, 2, 3, 3, 8),
                                           (736, 4, 3, 1, 5)])
def test_mixed_radix_solves(n, q, J, C, iters):
    w = make_small(n, q, J, channels=C, seed=n + q, lam=0.1, iters=iters)
    r, s, B, lam_f = run_oracle(w)
    g = run_gpu(w)
    assert np.max(np.abs(g["u"] - r.w)) < 2e-5
    assert np.mean(g["labels"] == r.labels) >= 0.999
    h = g["hist"]
    assert np.max(np.abs(h[:, 2] - r.r_combined) / r.r_combined) < 1e-3


def test_schedule_tuning_cached_and_described():
    # mixed-radix plans time their schedule candidates at creation; a second plan of the same
    # shape reuses the choice (process cache), so both give the same bits
    pkg = _pkg()
    w = make_small(352, 2, 3, seed=61, lam=0.1, iters=6)
    a = pkg.Plan(352, 1, 2, 3)
    b = pkg.Plan(352, 1, 2, 3)
    da, db = a.describe(), b.describe()
    print(da)
    assert "rows/wave" in da and ("tuned" in da or "cached" in da)
    assert "cached" in db and da.split(" (")[0] == db.split(" (")[0]
    assert "power-of-two" in pkg.Plan(256, 1, 2, 2).describe()
    outs = []
    for plan in (a, b):
        s = torch.empty((2, 352, 352), device="cuda:0")
        plan.datacost(dev_t(w.img), w.codebook, s)
        u = torch.empty_like(s)
        plan.solve(s, plan.new_workspace(), w.lam, w.gamma, w.iters, u=u)
        torch.cuda.synchronize()
        outs.append(u.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_unsupported_sizes_rejected():
    pkg = _pkg()
    for n in (100, 62, 1056, 2 * 29 * 8):
        with pytest.raises(pkg.ShsError) as e:
            pkg.Plan(n, 1, 2, 2)
        assert e.value.status == pkg.SHS_E_UNSUPPORTED


# ------------------------------------------------------------------ batches of images
def _batch_inputs(workloads, stores):
    pkg = _pkg()
    s_list, plans = [], []
    for w, st in zip(workloads, stores):
        plan = pkg.Plan(w.n, w.channels, w.q, w.J, st)
        s = torch.empty((w.q, w.n, w.n), dtype=torch.float32, device="cuda:0")
        plan.datacost(dev_t(w.img), w.codebook, s)
        s_list.append(s)
        plans.append(plan)
    return s_list, plans


def test_batch_equals_eager_solves_and_replays():
    from synth import make_c3_image
    pkg = _pkg()
    iters = 9
    ws_ = [make_c3_image(i) for i in (1, 4, 5)] + [make_small(128, 3, 2, channels=3, seed=2),
                                                   make_small(96, 5, 2, seed=3)]
    stores = ["f32", "f32", "bf16", "f16", "f32"]
    s_list, plans = _batch_inputs(ws_, stores)
    batch = pkg.Batch([(w.n, w.channels, w.q, w.J, st) for w, st in zip(ws_, stores)])
    bws = batch.new_workspace()
    lams = [w.lam for w in ws_]
    gammas = [w.gamma for w in ws_]
    eager = []
    for w, plan, s in zip(ws_, plans, s_list):
        u = torch.empty_like(s)
        lab = torch.empty((w.n, w.n), dtype=torch.int32, device="cuda:0")
        st = plan.solve(s, plan.new_workspace(), w.lam, w.gamma, iters, u=u, labels=lab)
        eager.append((u.cpu().numpy(), lab.cpu().numpy(), st))
    u_list = [torch.full_like(s, -1.0) for s in s_list]
    l_list = [torch.full((w.n, w.n), -1, dtype=torch.int32, device="cuda:0") for w in ws_]
    stats = torch.zeros((len(ws_), 5), dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        for u in u_list:
            u.fill_(-1.0)
        batch.solve(s_list, bws, lams, gammas, iters, u_list, l_list, stats)
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda:0").sum().item()
        for i, (eu, el, est) in enumerate(eager):
            assert np.array_equal(u_list[i].cpu().numpy(), eu), (rep, i)
            assert np.array_equal(l_list[i].cpu().numpy(), el), (rep, i)
        st = stats.cpu().numpy()
        for i, (_, _, est) in enumerate(eager):
            assert st[i, 4] == 0.0
            assert abs(np.sqrt(st[i, 1]) - est["r_primal"]) <= 1e-9 * max(1.0, est["r_primal"])
            assert abs(st[i, 2] + st[i, 3] - est["energy_surrogate"]) <= 1e-9 * abs(est["energy_surrogate"])
    del junk


def test_batch_oracle_parity_and_zero_iterations():
    from synth import make_c3_image
    pkg = _pkg()
    w = make_c3_image(1)      # 320 x 320, mixed-radix path
    iters = 10
    s_list, _ = _batch_inputs([w, make_small(64, 2, 1, seed=9)], ["f32", "f32"])
    batch = pkg.Batch([(w.n, 1, w.q, w.J, "f32"), (64, 1, 2, 1, "f32")])
    bws = batch.new_workspace()
    u_list = [torch.empty_like(s) for s in s_list]
    l_list = [torch.empty((s.shape[1], s.shape[2]), dtype=torch.int32, device="cuda:0") for s in s_list]
    batch.solve(s_list, bws, [w.lam, [0.0, 0.1]], [w.gamma, 1.0], iters, u_list, l_list)
    torch.cuda.synchronize()
    r, s, B, lam_f = run_oracle(w, iters=iters, s=f32(s_list[0].cpu().numpy()))
    assert np.max(np.abs(u_list[0].cpu().numpy() - r.w)) < 2e-5
    assert np.mean(l_list[0].cpu().numpy() == r.labels) >= 0.999
    # zero iterations: the zero start, and statistics rows of zeros (not stale workspace bytes)
    stats = torch.full((2, 5), float("nan"), dtype=torch.float64, device="cuda:0")
    batch.solve(s_list, bws, [w.lam, [0.0, 0.1]], [w.gamma, 1.0], 0, u_list, l_list, stats)
    torch.cuda.synchronize()
    assert all(torch.count_nonzero(u).item() == 0 for u in u_list)
    assert torch.count_nonzero(stats).item() == 0
    with pytest.raises(ValueError):
        batch.solve(s_list[:1] + [s_list[0]], bws, [w.lam, w.lam], [1.0, 1.0], 3)
