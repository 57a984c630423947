#!/usr/bin/env python3
"""Writes the stored ADMM results the full-length GPU parity tests compare against.

Every value in the files this script writes comes from the FP64 oracle (``oracle/``) run
on the seeded synthetic workloads of ``synth/``; nothing here reads the HIP library.
The oracle runs the ADMM of Section 3 literally (v, w, b_v, b_w; zero start; fixed
iteration count) on the float32 values the GPU sees (image and codebook rounded to
float32, then promoted to float64, exactly as the tests feed the oracle).

The full coefficient arrays of these sizes are too large to store, so each file keeps
what the tests compare:

* ``labels``       the label map argmax_k w^K (int8, [N][N]), Section 3's labelling;
* ``energy``       the exact energy F(w^K) of eq. (problemSegmentation);
* ``r_primal``, ``r_dual``, ``r_combined``, ``surrogate``: the per-iteration residual
  histories and energy surrogate, as the oracle defines them;
* ``sample_idx``, ``w_sample``: w^K at a fixed seeded sample of pixels, every label;
* ``w_label_sums`` the per-label sums of w^K;
* ``s_sum``, ``s_sq_sum``: checksums of the data term, so a change of the input
  generators is caught instead of being read as a parity failure.

Cases (the workload each one follows):

* ``c1``    512^2 gray, q=4, J=3, 500 iterations (the textured-regions workload);
* ``c2``    1024^2 RGB, q=5, J=4, 300 iterations (the precision-form workload);
* ``c4q3``  2048^2 gray, J=4 (61 filters), the large-instance image class with q=3
            grey levels, 12 iterations (q=8 needs ~45 GB of FP64 state in the oracle).
* ``c3``    nine images of the mixed-size batch workload at its full 200 iterations (FP32
            state on the GPU), one per FFT size class: sides 96, 160, 224, 256, 352, 416, 544,
            608 and 736 (largest prime factor of N/32: 3, 5, 7, 1, 11, 13, 17, 19, 23).  One
            file, the keys of image i prefixed ``i<i>_``.

Usage:  python tests/golden/make_admm_golden.py [c1 c2 c4q3 c3]     (default: all)
The oracle is run in chunks of iterations from the previous state (``init=``), which
equals one continuous run (pinned in tests/test_oracle_admm.py); the histories of the
chunks are concatenated.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import make_c1, make_c2, make_c4, make_c3_image  # noqa: E402

SAMPLE = 2048          # pixels whose w^K is stored (every label)
SAMPLE_SEED = 4242
CHUNK = 10             # iterations per oracle call (progress granularity)

CASES = {
    "c1": lambda: (make_c1(), None),
    "c2": lambda: (make_c2(), None),
    "c4q3": lambda: (make_c4(q=3), 12),
}
C3_IMAGES = (44, 24, 35, 17, 27, 2, 51, 0, 3)   # indices into the batch workload


def path_of(case: str) -> str:
    return os.path.join(HERE, f"admm_{case}.npz")


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def sample_indices(n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return np.sort(rng.choice(n * n, size=SAMPLE, replace=False)).astype(np.int64)


def solve(case: str, w, iters: int) -> dict:
    """The oracle's ADMM on workload w for `iters` iterations; the compact results."""
    t0 = time.time()
    s = O.datacost(f32(w.img), f32(w.codebook))
    bank = O.filter_bank(w.n, w.J)
    lam_f = O.lambda_per_filter(w.lam, w.J)
    print(f"{case}: n={w.n} q={w.q} J={w.J} eta={bank.shape[0]} iters={iters} gamma={w.gamma}", flush=True)
    res = None
    hist = {k: [] for k in ("r_primal", "r_dual", "r_combined", "surrogate")}
    done = 0
    while done < iters:
        k = min(CHUNK, iters - done)
        res = O.admm(s, bank, lam_f, w.gamma, k, init=res)
        for key in hist:
            hist[key].append(getattr(res, key))
        done += k
        print(f"  {case}: {done}/{iters} iterations, {time.time() - t0:.0f} s", flush=True)
    e = O.energy(res.w, s, bank, lam_f)
    idx = sample_indices(w.n)
    wf = res.w.reshape(w.q, -1)
    print(f"{case}: energy {e:.10g}, {time.time() - t0:.0f} s", flush=True)
    return dict(
        n=np.int64(w.n), q=np.int64(w.q), J=np.int64(w.J), iters=np.int64(iters),
        gamma=np.float64(w.gamma), lam=np.asarray(w.lam, dtype=np.float64),
        labels=res.labels.astype(np.int8), energy=np.float64(e),
        sample_idx=idx, w_sample=wf[:, idx].copy(), w_label_sums=wf.sum(axis=1),
        s_sum=np.float64(s.sum()), s_sq_sum=np.float64((s * s).sum()),
        **{k: np.concatenate(v) for k, v in hist.items()},
    )


def run_case(case: str) -> None:
    if case == "c3":
        out = {"case": np.array(case), "images": np.array(C3_IMAGES, dtype=np.int64)}
        for i in C3_IMAGES:
            w = make_c3_image(i)
            out.update({f"i{i}_{k}": v for k, v in solve(f"c3[{i}]", w, w.iters).items()})
    else:
        w, iters = CASES[case]()
        out = dict(case=np.array(case), **solve(case, w, w.iters if iters is None else iters))
    np.savez_compressed(path_of(case), **out)
    print(f"{case}: wrote {path_of(case)} ({os.path.getsize(path_of(case))} bytes)", flush=True)


def main(argv):
    known = list(CASES) + ["c3"]
    cases = argv or known
    for c in cases:
        if c not in known:
            raise SystemExit(f"unknown case {c}; known: {known}")
    for c in cases:
        run_case(c)


if __name__ == "__main__":
    main(sys.argv[1:])
