"""Meyer-type one-dimensional building blocks (Section 2, "Continuous Shearlets"
and "Shearlets on Cones").  Oracle: test infrastructure only.

All functions are vectorised over numpy arrays and evaluated in float64.
"""
from __future__ import annotations

import numpy as np


def meyer_v(x):
    """Auxiliary polynomial v of Section 2 (after eq. (psi1_psi2)):
    0 below 0, 35x^4 - 84x^5 + 70x^6 - 20x^7 on [0, 1], 1 above 1."""
    x = np.asarray(x, dtype=np.float64)
    poly = x ** 4 * (35.0 - 84.0 * x + 70.0 * x ** 2 - 20.0 * x ** 3)
    return np.where(x < 0.0, 0.0, np.where(x > 1.0, 1.0, poly))


def meyer_b(x):
    """Meyer profile b of Section 2: sin(pi/2 v(|x|-1)) for 1 <= |x| <= 2,
    cos(pi/2 v(|x|/2 - 1)) for 2 < |x| <= 4, and 0 otherwise."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    rise = np.sin(0.5 * np.pi * meyer_v(a - 1.0))
    fall = np.cos(0.5 * np.pi * meyer_v(0.5 * a - 1.0))
    return np.where((a >= 1.0) & (a <= 2.0), rise, np.where((a > 2.0) & (a <= 4.0), fall, 0.0))


def psi1_hat(w):
    """Radial window, eq. (psi1_psi2): sqrt(b^2(2w) + b^2(w)); support [-4,-1/2] u [1/2,4]."""
    w = np.asarray(w, dtype=np.float64)
    return np.sqrt(meyer_b(2.0 * w) ** 2 + meyer_b(w) ** 2)


def psi2_hat(w):
    """Angular bump, eq. (psi1_psi2): sqrt(v(1+w)) for w <= 0, sqrt(v(1-w)) for w > 0;
    support [-1, 1]."""
    w = np.asarray(w, dtype=np.float64)
    return np.where(w <= 0.0, np.sqrt(meyer_v(1.0 + w)), np.sqrt(meyer_v(1.0 - w)))


def phi_1d(w):
    """One-dimensional profile of the scaling function (Section 2, "Shearlets on Cones"):
    1 for |w| <= 1/2, cos(pi/2 v(2|w| - 1)) for 1/2 < |w| < 1, 0 otherwise."""
    a = np.abs(np.asarray(w, dtype=np.float64))
    mid = np.cos(0.5 * np.pi * meyer_v(2.0 * a - 1.0))
    return np.where(a <= 0.5, 1.0, np.where(a < 1.0, mid, 0.0))
