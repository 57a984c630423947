"""shs_solve_noalloc (the allocation-free solve) against shs_solve, through the C ABI.

Both entry points run the same kernels; the allocation-free one takes its workspace from
the library's per-GPU device array, so its outputs must equal shs_solve's bit for bit,
also on a second call with a smaller problem (the array then holds the larger problem's
leftovers, and the solve must start from its own zero state).
"""
import numpy as np
import pytest

import oracle as O
from synth import make_small

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pkg():
    import paper_1112_1805_amd as pkg
    pkg.lib()
    return pkg


def _inputs(pkg, w, store="f32"):
    plan = pkg.Plan(w.n, w.channels, w.q, w.J, store)
    s = torch.empty((w.q, w.n, w.n), dtype=torch.float32, device="cuda:0")
    plan.datacost(torch.tensor(np.float32(w.img), device="cuda:0"), w.codebook, s)
    return plan, s


def _solve_both(pkg, w, store="f32"):
    plan, s = _inputs(pkg, w, store)
    outs = []
    for noalloc in (False, True):
        u = torch.full((w.q, w.n, w.n), -1.0, device="cuda:0")
        lab = torch.full((w.n, w.n), -1, dtype=torch.int32, device="cuda:0")
        h = torch.zeros((w.iters, 4), dtype=torch.float64, device="cuda:0")
        if noalloc:
            st = plan.solve_noalloc(s, w.lam, w.gamma, w.iters, u=u, labels=lab, hist=h)
        else:
            st = plan.solve(s, plan.new_workspace(), w.lam, w.gamma, w.iters, u=u, labels=lab, hist=h)
        torch.cuda.synchronize()
        outs.append((u.cpu().numpy(), lab.cpu().numpy(), h.cpu().numpy(), st))
    return outs, plan, s


def test_noalloc_equals_solve_on_two_calls():
    pkg = _pkg()
    # first call: 128^2, q = 3, J = 2 (13 filters); second call: a smaller problem
    big = make_small(128, 3, 2, seed=41, lam=0.1, iters=15)
    small = make_small(64, 2, 1, seed=42, lam=0.15, iters=9)
    for w, store in ((big, "f32"), (small, "f16")):
        (ref, got), plan, s = _solve_both(pkg, w, store)
        assert plan.workspace_bytes() <= pkg.SHS_NOALLOC_MAX_BYTES
        assert np.array_equal(ref[0], got[0]), w.name
        assert np.array_equal(ref[1], got[1]), w.name
        assert np.array_equal(ref[2], got[2]), w.name
        assert ref[3] == got[3], w.name
    # the first problem's result also meets the oracle (same bar as the other ADMM tests)
    w = big
    (ref, got), plan, s = _solve_both(pkg, w)
    r = O.admm(O.datacost(np.float32(w.img).astype(np.float64), np.float32(w.codebook).astype(np.float64)),
               O.filter_bank(w.n, w.J), O.lambda_per_filter(w.lam, w.J), w.gamma, w.iters)
    assert np.max(np.abs(got[0] - r.w)) < 2e-5
    assert np.mean(got[1] == r.labels) >= 0.999


def test_noalloc_resume_and_size_limit():
    pkg = _pkg()
    w = make_small(128, 3, 2, seed=43, lam=0.1, iters=12)
    plan, s = _inputs(pkg, w)
    full = torch.empty((w.q, w.n, w.n), device="cuda:0")
    plan.solve_noalloc(s, w.lam, w.gamma, 12, u=full, want_stats=False)
    part = torch.empty_like(full)
    plan.solve_noalloc(s, w.lam, w.gamma, 7, u=part, want_stats=False)
    plan.solve_noalloc(s, w.lam, w.gamma, 5, u=part, want_stats=False, resume=True)
    torch.cuda.synchronize()
    assert torch.equal(full, part)
    # a plan whose workspace exceeds the array is rejected before any work
    huge = pkg.Plan(512, 1, 4, 3, "f32")
    assert huge.workspace_bytes() > pkg.SHS_NOALLOC_MAX_BYTES
    s2 = torch.zeros((4, 512, 512), device="cuda:0")
    with pytest.raises(pkg.ShsError) as e:
        huge.solve_noalloc(s2, [0.0, 0.1, 0.1, 0.1], 1.0, 2)
    assert e.value.status == pkg.SHS_E_WORKSPACE
