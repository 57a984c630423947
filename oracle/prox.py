"""Proximal maps of the v- and w-updates (Section 3: soft shrinkage and the pixelwise
orthogonal projection onto C).  Oracle: test infrastructure only.

Arrays of label vectors are laid out label-major: g[k, ...] is the k-th entry of the
label vector of every pixel, as in the layer layout of u of Section 3.
"""
from __future__ import annotations

import itertools

import numpy as np


def soft_shrink(x, t):
    """S_t(x) of Section 3: x - t for x > t, 0 on [-t, t], x + t for x < -t (t >= 0,
    broadcast against x)."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > t, x - t, np.where(x < -t, x + t, 0.0))


def project_simplex(g: np.ndarray) -> np.ndarray:
    """Euclidean projection of every label vector g[:, pixel] onto
    {x : x >= 0, sum_k x_k = 1} (the set C of Section 3, one pixel at a time).

    Sort-based evaluation of the projection (Held, Wolfe & Crowder 1974): with the
    entries sorted decreasingly, u_(1) >= ... >= u_(q), the threshold is
    tau = (sum_{i<=r} u_(i) - 1)/r for the largest r with u_(r) > tau_r; then
    x = max(g - tau, 0)."""
    g = np.asarray(g, dtype=np.float64)
    q = g.shape[0]
    u = -np.sort(-g, axis=0)
    css = np.cumsum(u, axis=0)
    r = np.arange(1, q + 1).reshape((q,) + (1,) * (g.ndim - 1))
    cond = u - (css - 1.0) / r > 0
    rho = q - np.argmax(cond[::-1], axis=0)            # largest r (1-based) with cond true
    tau = (np.take_along_axis(css, (rho - 1)[None], axis=0)[0] - 1.0) / rho
    return np.maximum(g - tau[None], 0.0)


def project_simplex_paper(g: np.ndarray, max_rounds: int | None = None) -> np.ndarray:
    """The projection as the paper describes it (end of Section 3): project onto the
    hyperplane <x, 1> = 1 by g + (1 - sum g)/q * 1; set the negative entries to zero and
    project again within the remaining coordinates; repeat until nothing is negative."""
    g = np.asarray(g, dtype=np.float64)
    q = g.shape[0]
    active = np.ones(g.shape, dtype=bool)
    x = np.zeros_like(g)
    for _ in range(max_rounds or q):
        cnt = active.sum(axis=0)
        shift = (1.0 - np.where(active, g, 0.0).sum(axis=0)) / cnt
        x = np.where(active, g + shift[None], 0.0)
        neg = active & (x < 0)
        if not neg.any():
            return x
        active &= ~neg
    return x


def project_simplex_bruteforce(g: np.ndarray) -> np.ndarray:
    """Projection by enumeration of all 2^q - 1 supports (tiny q only): on every support
    A take the projection onto the affine hull {x_A : sum x_A = 1}, keep it if it is
    feasible, and return the feasible candidate nearest to g."""
    g = np.asarray(g, dtype=np.float64)
    q = g.shape[0]
    flat = g.reshape(q, -1)
    out = np.empty_like(flat)
    for p in range(flat.shape[1]):
        gp = flat[:, p]
        best, best_d = None, np.inf
        for size in range(1, q + 1):
            for A in itertools.combinations(range(q), size):
                A = list(A)
                x = np.zeros(q)
                x[A] = gp[A] - (gp[A].sum() - 1.0) / size
                if np.all(x >= 0):
                    d = np.sum((x - gp) ** 2)
                    if d < best_d:
                        best, best_d = x, d
        out[:, p] = best
    return out.reshape(g.shape)
