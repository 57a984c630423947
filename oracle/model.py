"""Convex multi-label segmentation model and its ADMM (Section 3).  Oracle: test
infrastructure only.

The iteration is run literally, with the four arrays v, w, b_v, b_w of the paper's
ADMM for (problemSegmentationADMM):

    u^{i+1} = 1/2 [ (I_q (x) S)^T (v^i - b_v^i) + (w^i - b_w^i) - gamma s ]
    v^{i+1} = S_{gamma Lambda}( b_v^i + (I_q (x) S) u^{i+1} )      (soft shrinkage)
    w^{i+1} = P_C( b_w^i + u^{i+1} )                                (pixelwise simplex)
    b_v^{i+1} = b_v^i + (I_q (x) S) u^{i+1} - v^{i+1}
    b_w^{i+1} = b_w^i + u^{i+1} - w^{i+1}

Readings (the paper leaves them open): v^0 = w^0 = b^0 = 0; a fixed number of
iterations; the threshold of a filter of scale j is gamma * lambda_{j+1}, the
low-pass uses gamma * lambda_0; the relaxed result is w^K (which lies in C) and the
label of a pixel is the index of its largest entry, lowest index on ties (0-based).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .filters import filter_scale_index, num_filters
from .prox import project_simplex, soft_shrink
from .transform import adjoint, forward


def datacost(img: np.ndarray, codebook: np.ndarray, p: float = 2.0) -> np.ndarray:
    """Data term s of eq. (computationOfs): s[k] = ||f - c_k||_p^p per pixel; for a
    colour image the norm is taken over the channel vector (RGB paragraph of Section 4).

    img [C][N][N], codebook [q][C]  ->  s [q][N][N]."""
    img = np.asarray(img, dtype=np.float64)
    cb = np.asarray(codebook, dtype=np.float64)
    diff = img[None, :, :, :] - cb[:, :, None, None]
    return np.sum(np.abs(diff) ** p, axis=1)


def lambda_per_filter(lam, J: int) -> np.ndarray:
    """Expand Lambda = (lambda_0, .., lambda_J) (one weight per scale, the low-pass
    first; Section 3) to one weight per filter.  A vector of length eta is taken as
    already per filter (the paper allows per-shear weights)."""
    lam = np.asarray(lam, dtype=np.float64).ravel()
    eta = num_filters(J)
    if lam.size == eta and eta != J + 1:
        return lam.copy()
    if lam.size != J + 1:
        raise ValueError(f"Lambda needs J+1={J + 1} or eta={eta} entries, got {lam.size}")
    return lam[filter_scale_index(J)]


def labels_of(u: np.ndarray) -> np.ndarray:
    """Label map: index of the largest layer entry per pixel (Section 3), lowest index
    first on ties, 0-based."""
    return np.argmax(u, axis=0).astype(np.int32)


def energy(w: np.ndarray, s: np.ndarray, bank: np.ndarray, lam_f: np.ndarray) -> float:
    """F(w) = <w, s> + ||Lambda (I_q (x) S) w||_1 of eq. (problemSegmentation), for w in C."""
    e = float(np.sum(w * s))
    for l in range(w.shape[0]):
        c = forward(w[l], bank)
        e += float(np.sum(lam_f[:, None, None] * np.abs(c)))
    return e


@dataclass
class AdmmResult:
    u: np.ndarray          # u^K                [q][N][N]
    v: np.ndarray          # v^K                [q][eta][N][N]
    w: np.ndarray          # w^K (relaxed result, in C)
    b_v: np.ndarray
    b_w: np.ndarray
    labels: np.ndarray     # argmax of w^K      [N][N] int32
    r_primal: np.ndarray   # ||b^{i+1} - b^i||                 per iteration
    r_dual: np.ndarray     # ||y^{i+1} - y^i|| / gamma, y=(v,w) per iteration
    r_combined: np.ndarray  # ||y^{i+1}-y^i||^2 + ||b^{i+1}-b^i||^2
    surrogate: np.ndarray  # <w^i, s> + sum lambda |v^i|        per iteration


def admm(s: np.ndarray, bank: np.ndarray, lam_f: np.ndarray, gamma: float, iters: int,
         init: AdmmResult | None = None) -> AdmmResult:
    """Run `iters` ADMM iterations for (problemSegmentationADMM) from the zero state
    (or from `init`).  s [q][N][N]; bank [eta][N][N]; lam_f [eta] (per-filter weights)."""
    s = np.asarray(s, dtype=np.float64)
    q, n, _ = s.shape
    eta = bank.shape[0]
    thr = (gamma * np.asarray(lam_f, dtype=np.float64))[:, None, None]
    if init is None:
        v = np.zeros((q, eta, n, n))
        b_v = np.zeros((q, eta, n, n))
        w = np.zeros((q, n, n))
        b_w = np.zeros((q, n, n))
        u = np.zeros((q, n, n))
    else:
        v, b_v, w, b_w, u = (init.v.copy(), init.b_v.copy(), init.w.copy(), init.b_w.copy(),
                             init.u.copy())
    rp, rd, rc, sur = [], [], [], []
    for _ in range(iters):
        # u-update: A^T A = 2I (eq. (important)), so u is the closed form above.
        for l in range(q):
            u[l] = 0.5 * (adjoint(v[l] - b_v[l], bank) + (w[l] - b_w[l]) - gamma * s[l])
        db2 = dy2 = 0.0
        l1 = 0.0
        for l in range(q):
            Su = forward(u[l], bank)
            g_v = b_v[l] + Su
            v_new = soft_shrink(g_v, thr)
            b_v_new = g_v - v_new
            dy2 += float(np.sum((v_new - v[l]) ** 2))
            db2 += float(np.sum((b_v_new - b_v[l]) ** 2))
            l1 += float(np.sum(np.asarray(lam_f)[:, None, None] * np.abs(v_new)))
            v[l], b_v[l] = v_new, b_v_new
        g_w = b_w + u
        w_new = project_simplex(g_w)
        b_w_new = g_w - w_new
        dy2 += float(np.sum((w_new - w) ** 2))
        db2 += float(np.sum((b_w_new - b_w) ** 2))
        w, b_w = w_new, b_w_new
        rp.append(np.sqrt(db2))
        rd.append(np.sqrt(dy2) / gamma)
        rc.append(dy2 + db2)
        sur.append(float(np.sum(w * s)) + l1)
    return AdmmResult(u=u, v=v, w=w, b_v=b_v, b_w=b_w, labels=labels_of(w),
                      r_primal=np.array(rp), r_dual=np.array(rd), r_combined=np.array(rc),
                      surrogate=np.array(sur))
