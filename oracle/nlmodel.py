"""Nonlocal (NL-means graph) regulariser of Section 4 and a primal-dual solver for the
segmentation model with it.  Oracle: test infrastructure only.

Graph (Section 4): for every pixel i (row-major order) and every j != i in the
search window of side `window` around i, the patch distance

    d_a(i, j) = sum_{t1, t2 in [-h, h]} G_a(t1, t2) (f(i + t) - f(j + t))^2,   h = (p-1)/2,

with G_a the normalised Gaussian of standard deviation a on the p x p patch.  With l the
number of nonzero weights w(i, .) already set when i is reached, i picks
k = min(m, 2m - l) neighbours j of smallest distance and sets w(i, j) = w(j, i) = 1.
D (m_blocks = 2m blocks of N^2 rows) has in block b the row -e_i + e_{j_b(i)} for the
b-th neighbour j_b(i) of i, and a zero row if i has fewer than b + 1 neighbours.
The regulariser replaces grad by D in the coupled TV: sum_i (sum_l sum_b (D_b u_l)(i)^2)^(1/2).

Readings (the paper leaves them open): periodic image boundary for windows and
patches; colour images sum the patch distance over the channels; a candidate j is
eligible if w(i, j) = 0 and j has fewer than 2m nonzero weights (so no pixel exceeds the
2m rows of D), ties go to the smaller linear index, the neighbour order of a pixel is the
order in which its weights were set; the model is solved by the primal-dual iteration
(Chambolle & Pock, theta = 1) since (I + D^T D) is not diagonalised by the DFT:

    y = P_ball(y + sigma K ubar)      (per pixel over labels and blocks, radius lambda)
    u' = P_C(u - tau (K^T y + s)),  ubar = 2 u' - u,   K = I_q (x) D,

with sigma tau ||K||^2 <= 1; ||D||^2 <= ||D||_1 ||D||_inf = 2 * 2 max-degree.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .model import labels_of
from .prox import project_simplex


def gaussian_patch(p: int, a: float) -> np.ndarray:
    """Normalised p x p Gaussian G_a (standard deviation a), centred."""
    h = (p - 1) // 2
    t = np.arange(-h, h + 1, dtype=np.float64)
    g = np.exp(-(t[:, None] ** 2 + t[None, :] ** 2) / (2.0 * a * a))
    return g / np.sum(g)


def patch_distance(img: np.ndarray, i: tuple, j: tuple, G: np.ndarray) -> float:
    """d_a(i, j) of one pixel pair, by the definition (periodic boundary); img [C][N][N]."""
    C, n, _ = img.shape
    h = (G.shape[0] - 1) // 2
    d = 0.0
    for t1 in range(-h, h + 1):
        for t2 in range(-h, h + 1):
            for c in range(C):
                diff = img[c, (i[0] + t1) % n, (i[1] + t2) % n] - img[c, (j[0] + t1) % n, (j[1] + t2) % n]
                d += G[t1 + h, t2 + h] * (diff * diff)
    return d


def window_distances(img: np.ndarray, p: int, window: int, a: float):
    """All d_a(i, i + o) for the window offsets o != 0: returns (offsets [K][2], D [K][N][N])
    with D[k][i] = d_a(i, i + offsets[k]) (vectorised over pixels, same sum order as
    patch_distance: t1, t2, channel)."""
    img = np.asarray(img, dtype=np.float64)
    C, n, _ = img.shape
    G = gaussian_patch(p, a)
    h = (p - 1) // 2
    r = (window - 1) // 2
    offs = [(o1, o2) for o1 in range(-r, r + 1) for o2 in range(-r, r + 1) if (o1, o2) != (0, 0)]
    out = np.zeros((len(offs), n, n))
    for k, (o1, o2) in enumerate(offs):
        acc = np.zeros((n, n))
        for t1 in range(-h, h + 1):
            for t2 in range(-h, h + 1):
                for c in range(C):
                    a_img = np.roll(img[c], (-t1, -t2), axis=(0, 1))             # f(i + t)
                    b_img = np.roll(img[c], (-(t1 + o1), -(t2 + o2)), axis=(0, 1))   # f(i + o + t)
                    diff = a_img - b_img
                    acc = acc + G[t1 + h, t2 + h] * (diff * diff)
        out[k] = acc
    return np.array(offs), out


def nl_graph(img: np.ndarray, p: int = 5, window: int = 15, a: float = 2.0, m: int = 5) -> np.ndarray:
    """Neighbour lists of the paper's construction: nbr [2m][N][N] int64 (linear index of
    the b-th neighbour, -1 if none)."""
    img = np.asarray(img, dtype=np.float64)
    n = img.shape[-1]
    assert n >= window, "the search window must fit in the image (no wrapped duplicates)"
    offs, dist = window_distances(img, p, window, a)
    nbrs = [[] for _ in range(n * n)]
    for i in range(n * n):
        r0, c0 = divmod(i, n)
        l = len(nbrs[i])
        k = min(m, 2 * m - l)
        if k <= 0:
            continue
        cand = []
        for kk, (o1, o2) in enumerate(offs):
            j = ((r0 + o1) % n) * n + (c0 + o2) % n
            if j == i or j in nbrs[i] or len(nbrs[j]) >= 2 * m:
                continue
            cand.append((dist[kk, r0, c0], j))
        cand.sort()
        for d, j in cand[:k]:
            nbrs[i].append(j)
            nbrs[j].append(i)
    out = -np.ones((2 * m, n, n), dtype=np.int64)
    for i in range(n * n):
        for b, j in enumerate(nbrs[i]):
            out[b, i // n, i % n] = j
    return out


def apply_D(u: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """D u for u [N][N]: [2m][N][N], row (b, i) = u(j_b(i)) - u(i) or 0."""
    flat = u.ravel()
    nb = nbr.reshape(nbr.shape[0], -1)
    val = np.where(nb >= 0, flat[np.maximum(nb, 0)] - flat[None, :], 0.0)
    return val.reshape(nbr.shape)


def apply_Dt(y: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """D^T y for y [2m][N][N] -> [N][N] (scatter form of the transpose)."""
    n = nbr.shape[-1]
    nb = nbr.reshape(nbr.shape[0], -1)
    yy = y.reshape(y.shape[0], -1)
    out = np.zeros(n * n)
    for b in range(nb.shape[0]):
        ok = nb[b] >= 0
        np.add.at(out, nb[b][ok], yy[b][ok])
        out[ok] -= yy[b][ok]
    return out.reshape(n, n)


def nl_tv(u: np.ndarray, nbr: np.ndarray) -> float:
    """sum_i (sum_l sum_b (D_b u_l)(i)^2)^(1/2) for u [q][N][N]."""
    g = np.stack([apply_D(u[l], nbr) for l in range(u.shape[0])])
    return float(np.sum(np.sqrt(np.sum(g * g, axis=(0, 1)))))


def nl_energy(u: np.ndarray, s: np.ndarray, nbr: np.ndarray, lam: float) -> float:
    return float(np.sum(u * s)) + lam * nl_tv(u, nbr)


@dataclass
class NlResult:
    u: np.ndarray
    y: np.ndarray          # [q][2m][N][N]
    labels: np.ndarray
    du: np.ndarray         # ||u' - u|| per iteration
    dy: np.ndarray         # ||y' - y|| per iteration
    surrogate: np.ndarray  # <u', s> + lambda sum_i ||(K ubar)(i)|| per iteration


def nl_primal_dual(s: np.ndarray, nbr: np.ndarray, lam: float, tau: float, sigma: float, iters: int) -> NlResult:
    """Primal-dual iterations for min <u, s> + lambda NL-TV(u) + iota_C(u) from zero."""
    s = np.asarray(s, dtype=np.float64)
    q, n, _ = s.shape
    mb = nbr.shape[0]
    u = np.zeros((q, n, n))
    ubar = np.zeros((q, n, n))
    y = np.zeros((q, mb, n, n))
    du, dy, sur = [], [], []
    for _ in range(iters):
        ku = np.stack([apply_D(ubar[l], nbr) for l in range(q)])
        z = y + sigma * ku
        norm = np.sqrt(np.sum(z * z, axis=(0, 1)))
        y_new = z * np.minimum(1.0, lam / np.where(norm > 0, norm, 1.0))[None, None]
        kty = np.stack([apply_Dt(y_new[l], nbr) for l in range(q)])
        u_new = project_simplex(u - tau * (kty + s))
        du.append(float(np.sqrt(np.sum((u_new - u) ** 2))))
        dy.append(float(np.sqrt(np.sum((y_new - y) ** 2))))
        sur.append(float(np.sum(u_new * s)) + lam * float(np.sum(np.sqrt(np.sum(ku * ku, axis=(0, 1))))))
        ubar = 2.0 * u_new - u
        u, y = u_new, y_new
    return NlResult(u=u, y=y, labels=labels_of(u), du=np.array(du), dy=np.array(dy), surrogate=np.array(sur))
