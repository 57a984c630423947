"""First-order primal-dual iteration for the segmentation model of Section 3 (the
alternative to the ADMM that the paper names at the end of Section 3, Chambolle & Pock's
method).  Oracle: test infrastructure only.

The model (problemSegmentation) is  min_u <u, s> + iota_C(u) + ||Lambda (I_q (x) S) u||_1.
With K = I_q (x) S, G(u) = <u, s> + iota_C(u) and F(c) = sum_j lambda_j ||c_j||_1, the
iteration of Chambolle & Pock (2011, Algorithm 1, extrapolation theta = 1) reads

    y^{n+1} = prox_{sigma F*}(y^n + sigma K ubar^n)   = clip(y^n + sigma K ubar^n, +-lambda_j)
    u^{n+1} = prox_{tau G}(u^n - tau K^T y^{n+1})     = P_C(u^n - tau (K^T y^{n+1} + s))
    ubar^{n+1} = 2 u^{n+1} - u^n

(F* is the indicator of the box |y_j| <= lambda_j, so its prox is a clip; the prox of G
is the pixelwise projection onto the simplex C of the shifted point).  The shearlets are
a Parseval frame (Theorem 2.2), so ||K|| = 1 and sigma * tau <= 1 is the step condition.

Readings (the paper states no primal-dual details): zero start u = ubar = y = 0; a fixed
number of iterations; the result is u^K (it lies in C); labels as for the ADMM.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .model import energy, labels_of
from .prox import project_simplex
from .transform import adjoint, forward


@dataclass
class PdResult:
    u: np.ndarray          # u^K                 [q][N][N] (in C)
    ubar: np.ndarray       # 2 u^K - u^{K-1}
    y: np.ndarray          # y^K                 [q][eta][N][N]
    labels: np.ndarray     # argmax of u^K       [N][N] int32
    du: np.ndarray         # ||u^{n+1} - u^n||   per iteration
    dy: np.ndarray         # ||y^{n+1} - y^n||   per iteration
    surrogate: np.ndarray  # <u^{n+1}, s> + sum_j lambda_j ||(K ubar^n)_j||_1 per iteration
    gap: np.ndarray        # P(u^{n+1}) - D(y^{n+1}) per iteration (empty unless asked)


def dual_value(y: np.ndarray, s: np.ndarray, bank: np.ndarray) -> float:
    """D(y) = min_{u in C} <u, s + K^T y> - F*(y) for y in the box (F*(y) = 0): the
    minimum over the simplex of a linear function is its smallest coefficient, per pixel."""
    t = np.stack([s[l] + adjoint(y[l], bank) for l in range(s.shape[0])])
    return float(np.sum(np.min(t, axis=0)))


def primal_dual(s: np.ndarray, bank: np.ndarray, lam_f: np.ndarray, tau: float, sigma: float, iters: int,
                with_gap: bool = False) -> PdResult:
    """Run `iters` primal-dual iterations from the zero state.  s [q][N][N]; bank
    [eta][N][N]; lam_f [eta] per-filter weights; tau, sigma > 0 with tau * sigma <= 1."""
    s = np.asarray(s, dtype=np.float64)
    q, n, _ = s.shape
    eta = bank.shape[0]
    lam = np.asarray(lam_f, dtype=np.float64)[:, None, None]
    u = np.zeros((q, n, n))
    ubar = np.zeros((q, n, n))
    y = np.zeros((q, eta, n, n))
    du, dy, sur, gap = [], [], [], []
    for _ in range(iters):
        dy2 = 0.0
        l1 = 0.0
        for l in range(q):
            c = forward(ubar[l], bank)                      # K ubar
            y_new = np.clip(y[l] + sigma * c, -lam, lam)    # prox of sigma F*
            dy2 += float(np.sum((y_new - y[l]) ** 2))
            l1 += float(np.sum(lam * np.abs(c)))
            y[l] = y_new
        kty = np.stack([adjoint(y[l], bank) for l in range(q)])
        u_new = project_simplex(u - tau * (kty + s))        # prox of tau G
        du.append(np.sqrt(float(np.sum((u_new - u) ** 2))))
        dy.append(np.sqrt(dy2))
        sur.append(float(np.sum(u_new * s)) + l1)
        ubar = 2.0 * u_new - u
        u = u_new
        if with_gap:
            gap.append(energy(u, s, bank, np.asarray(lam_f, dtype=np.float64)) - dual_value(y, s, bank))
    return PdResult(u=u, ubar=ubar, y=y, labels=labels_of(u), du=np.array(du), dy=np.array(dy),
                    surrogate=np.array(sur), gap=np.array(gap))
