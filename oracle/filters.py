"""Finite discrete shearlet filter bank (Section 2, "Finite Discrete Shearlets",
Theorem 2.2).  Oracle: test infrastructure only.

Filter order (a convention of this project, used by every caller):

    0                       low-pass  phi_hat(xi) = phi(||xi||_inf)
    then for scale j = 0 .. J-1:
        2^(j+1)-1 filters   horizontal cone, shear k = -(2^j-1) .. 2^j-1
        2^(j+1)-1 filters   vertical cone,   shear k = -(2^j-1) .. 2^j-1
        2 filters           glued seam filters, k = -2^j then k = +2^j

so eta = 1 + 4 (2^J - 1) filters: 5, 13, 29, 61 for J = 1..4 (the paper's
"61 images" for four scales, Remark 2.3).

Frequencies.  FFT index n in [0, N) stands for omega = n for n < ceil(N/2) and
omega = n - N otherwise, i.e. the set Omega of Section 2.  The paper evaluates
psi1_hat(4^-j omega_1) on the integer grid with j_0 = floor(log2(N)/2) scales;
with a number of scales J chosen independently of N, the J-scale radial
partition sum_j psi1_hat(4^-j x)^2 + phi(x)^2 = 1 holds for |x| <= 2^(2J-1)
only.  Reading: evaluate at xi = rho * omega with rho = 4^J / N, so that the
largest grid frequency |omega| = N/2 lands exactly on 2^(2J-1).  For N = 4^J
this is the paper's integer grid.
"""
from __future__ import annotations

import numpy as np

from .meyer import phi_1d, psi1_hat, psi2_hat


def freq_index(n: int) -> np.ndarray:
    """Map FFT index 0..N-1 to the integer frequency of Omega (Section 2)."""
    idx = np.arange(n)
    return np.where(idx < (n + 1) // 2, idx, idx - n).astype(np.int64)


def num_filters(J: int) -> int:
    """eta = 1 + sum_{j<J} 2^(j+2): one low-pass plus, per scale j, 2(2^(j+1)-1) cone
    filters and 2 seam filters (Theorem 2.2's system)."""
    return 1 + 4 * (2 ** J - 1)


def filter_list(J: int) -> list[tuple[str, int, int]]:
    """(kind, scale j, shear k) for every filter, in the project's filter order."""
    out = [("low", -1, 0)]
    for j in range(J):
        ks = range(-(2 ** j - 1), 2 ** j)
        out += [("h", j, k) for k in ks]
        out += [("v", j, k) for k in ks]
        out += [("seam", j, -(2 ** j)), ("seam", j, 2 ** j)]
    return out


def filter_scale_index(J: int) -> np.ndarray:
    """sigma(filter): 0 for the low-pass, j+1 for a filter of scale j (the index into
    Lambda = (lambda_0, lambda_1, .., lambda_J) of Section 3)."""
    return np.array([0 if kind == "low" else j + 1 for kind, j, _ in filter_list(J)], dtype=np.int64)


def _cone_h(xi1, xi2, j, k):
    """psi1_hat(4^-j xi1) psi2_hat(2^j xi2/xi1 + k): the discrete shearlet of Section 2
    for the horizontal cone, evaluated where xi1 != 0."""
    safe = np.where(xi1 == 0.0, 1.0, xi1)
    return psi1_hat(xi1 / 4.0 ** j) * psi2_hat(2.0 ** j * xi2 / safe + k)


def eval_filter(kind: str, j: int, k: int, om1: np.ndarray, om2: np.ndarray, rho: float) -> np.ndarray:
    """Value of one filter at integer frequencies (om1, om2) (broadcast arrays)."""
    a1, a2 = np.abs(om1), np.abs(om2)
    xi1 = rho * om1.astype(np.float64)
    xi2 = rho * om2.astype(np.float64)
    cone_h = a2 < a1            # C^h (the |omega_1| >= 1/2 part is implied by psi1's support)
    cone_v = a1 < a2            # C^v
    diag = (a1 == a2) & (a1 > 0)  # C^x, the seam lines
    if kind == "low":
        # phi_hat(w) = phi(w_1) on |w_2| <= |w_1| and phi(w_2) on |w_1| < |w_2|, i.e. phi(||w||_inf).
        return phi_1d(np.maximum(np.abs(xi1), np.abs(xi2)))
    h = np.where(cone_h, _cone_h(xi1, xi2, j, k), 0.0)
    v = np.where(cone_v, _cone_h(xi2, xi1, j, k), 0.0)
    if kind == "h":
        return h
    if kind == "v":
        return v
    if kind == "seam":
        # Glued seam shearlet psi^h + psi^v + psi^x for |k| = 2^j; on the diagonal the
        # horizontal formula is used (psi_hat restricted to C^x).
        x = np.where(diag, _cone_h(xi1, xi2, j, k), 0.0)
        return h + v + x
    raise ValueError(kind)


def filter_bank(n: int, J: int, symmetrize_nyquist: bool = True) -> np.ndarray:
    """All eta filters on the full N x N FFT grid, float64 [eta][N][N], axis 0 <-> omega_1.

    For even N the bins with omega_1 = -N/2 or omega_2 = -N/2 have no mirror partner
    inside Omega; there the shear filters are not symmetric, which would make the
    coefficients complex, while Section 3 treats them as real.  Reading: replace the
    value there by sqrt((psi(w)^2 + psi(w_bar)^2)/2), w_bar = -w mod N, which keeps
    sum_j psi_j^2 = 1 (Theorem 2.2) bin by bin.
    """
    if J < 1:
        raise ValueError("J >= 1")
    om = freq_index(n)
    om1 = om[:, None]
    om2 = om[None, :]
    rho = 4.0 ** J / n
    bank = np.stack([eval_filter(kind, j, k, om1, om2, rho) for kind, j, k in filter_list(J)])
    if symmetrize_nyquist and n % 2 == 0:
        mirror = (-np.arange(n)) % n
        bar = bank[:, mirror, :][:, :, mirror]
        idx = np.arange(n)
        mask = (idx[:, None] == n // 2) | (idx[None, :] == n // 2)
        sym = np.sqrt(0.5 * (bank ** 2 + bar ** 2))
        bank = np.where(mask[None], sym, bank)
    return bank
