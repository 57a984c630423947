"""TV-regularised multi-label model (the comparison model of Section 4) and an ADMM for it.
Oracle: test infrastructure only.

Section 4 compares the shearlet model with the same data term and the TV regulariser of
Lellmann et al., coupled over the labels:

    TV(u) = sum_pixels ( |grad u_1|^2 + ... + |grad u_q|^2 )^(1/2),
    min_u  <u, s> + lambda TV(u) + iota_C(u).

The paper states no solver for it.  Readings: the discrete gradient is the forward
difference with periodic boundaries (so grad^T grad is diagonalised by the DFT), and the
solver is the ADMM of Section 3 with grad in place of S, A = [I_q (x) grad; I]:

    u^{i+1} = (I + grad^T grad)^{-1} [ grad^T (v^i - b_v^i) + (w^i - b_w^i) - gamma s ]
    v^{i+1} = shrink_{gamma lambda}(b_v^i + grad u^{i+1})   (per pixel, on the 2q-vector)
    w^{i+1} = P_C(b_w^i + u^{i+1})
    b_v^{i+1} = b_v^i + grad u^{i+1} - v^{i+1},   b_w^{i+1} = b_w^i + u^{i+1} - w^{i+1}

(A^T A = I + grad^T grad per label; the isotropic shrinkage is the prox of the coupled
norm: x * max(1 - t / ||x||, 0) over all labels and both directions of a pixel).  Zero
start, fixed iteration count, result w^K, labels as for the shearlet model.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .model import labels_of
from .prox import project_simplex
from .transform import fft2, ifft2


def grad(u: np.ndarray) -> np.ndarray:
    """Forward differences with periodic boundaries: [..][N][N] -> [..][2][N][N]
    (component 0 along axis -2, component 1 along axis -1)."""
    return np.stack([np.roll(u, -1, axis=-2) - u, np.roll(u, -1, axis=-1) - u], axis=-3)


def grad_adjoint(p: np.ndarray) -> np.ndarray:
    """grad^T p = -div p for p [..][2][N][N] -> [..][N][N]."""
    return (np.roll(p[..., 0, :, :], 1, axis=-2) - p[..., 0, :, :]) + \
           (np.roll(p[..., 1, :, :], 1, axis=-1) - p[..., 1, :, :])


def tv(u: np.ndarray) -> float:
    """Coupled isotropic TV of u [q][N][N]."""
    g = grad(u)                                   # [q][2][N][N]
    return float(np.sum(np.sqrt(np.sum(g * g, axis=(0, 1)))))


def tv_energy(u: np.ndarray, s: np.ndarray, lam: float) -> float:
    """<u, s> + lambda TV(u) (the indicator of C is not evaluated)."""
    return float(np.sum(u * s)) + lam * tv(u)


def solve_identity_plus_laplacian(r: np.ndarray) -> np.ndarray:
    """(I + grad^T grad) u = r for r [N][N]: with periodic forward differences grad^T grad
    has the DFT eigenvalues 4 sin^2(pi k0 / N) + 4 sin^2(pi k1 / N)."""
    n = r.shape[-1]
    e = 4.0 * np.sin(np.pi * np.arange(n) / n) ** 2
    return ifft2(fft2(r) / (1.0 + e[:, None] + e[None, :])).real


def group_shrink(g: np.ndarray, t: float) -> np.ndarray:
    """prox of t ||.||_2 over the label and direction axes of every pixel: g [q][2][N][N]."""
    norm = np.sqrt(np.sum(g * g, axis=(0, 1)))
    scale = np.where(norm > t, 1.0 - t / np.where(norm > 0, norm, 1.0), 0.0)
    return g * scale[None, None]


@dataclass
class TvResult:
    u: np.ndarray
    v: np.ndarray          # [q][2][N][N]
    w: np.ndarray          # relaxed result (in C)
    b_v: np.ndarray
    b_w: np.ndarray
    labels: np.ndarray
    r_primal: np.ndarray   # ||b^{i+1} - b^i||
    r_dual: np.ndarray     # ||y^{i+1} - y^i|| / gamma, y = (v, w)
    r_combined: np.ndarray
    surrogate: np.ndarray  # <w^i, s> + lambda sum_pixels ||v^i(pixel)||


def tv_admm(s: np.ndarray, lam: float, gamma: float, iters: int) -> TvResult:
    """Run `iters` ADMM iterations for the TV model from the zero state; s [q][N][N]."""
    s = np.asarray(s, dtype=np.float64)
    q, n, _ = s.shape
    v = np.zeros((q, 2, n, n))
    b_v = np.zeros((q, 2, n, n))
    w = np.zeros((q, n, n))
    b_w = np.zeros((q, n, n))
    u = np.zeros((q, n, n))
    rp, rd, rc, sur = [], [], [], []
    for _ in range(iters):
        for l in range(q):
            u[l] = solve_identity_plus_laplacian(grad_adjoint(v[l] - b_v[l]) + (w[l] - b_w[l]) - gamma * s[l])
        g_v = b_v + grad(u)
        v_new = group_shrink(g_v, gamma * lam)
        b_v_new = g_v - v_new
        g_w = b_w + u
        w_new = project_simplex(g_w)
        b_w_new = g_w - w_new
        dy2 = float(np.sum((v_new - v) ** 2) + np.sum((w_new - w) ** 2))
        db2 = float(np.sum((b_v_new - b_v) ** 2) + np.sum((b_w_new - b_w) ** 2))
        v, b_v, w, b_w = v_new, b_v_new, w_new, b_w_new
        rp.append(np.sqrt(db2))
        rd.append(np.sqrt(dy2) / gamma)
        rc.append(dy2 + db2)
        sur.append(float(np.sum(w * s)) + lam * float(np.sum(np.sqrt(np.sum(v * v, axis=(0, 1))))))
    return TvResult(u=u, v=v, w=w, b_v=b_v, b_w=b_w, labels=labels_of(w), r_primal=np.array(rp),
                    r_dual=np.array(rd), r_combined=np.array(rc), surrogate=np.array(sur))
