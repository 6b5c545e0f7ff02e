"""Oracle: the rotationally invariant kernel of Eq. 10 (test infrastructure only).

b(x) = sum_{l=0}^{lmax} (2l+1)/(4 pi) b_l P_l(x), evaluated by direct summation
for every requested argument.  The argument is passed as y = 1 - x = 1 - cos(gamma)
and the Legendre recurrence is run in y, so that pairs a fraction of a pixel
apart keep full relative precision (forming x first would round 1 - x to about
1e-16 absolute, which at lmax = 3000 is 1e-10 of the beam's width in x).
"""
from __future__ import annotations

import numpy as np


def legendre_series_in_y(coef_l, y):
    """sum_l c_l P_l(1 - y) with c_l = (2l+1) coef_l / (4 pi)   (Eq. 10).

    Recurrence in y with D_l = P_l - P_{l-1}:
        P_0 = 1, D_1 = -y, (l+1) D_{l+1} = l D_l - (2l+1) y P_l, P_{l+1} = P_l + D_{l+1}.
    """
    coef_l = np.asarray(coef_l, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    lmax = coef_l.shape[0] - 1
    c = (2.0 * np.arange(lmax + 1) + 1.0) * coef_l / (4.0 * np.pi)
    p = np.ones_like(y)
    acc = c[0] * p
    d = -y
    for l in range(0, lmax):
        if l > 0:
            d = (l * d - (2 * l + 1) * y * p) / (l + 1)
        p = p + d
        acc = acc + c[l + 1] * p
    return acc


def legendre_series_in_x(coef_l, x):
    """The same sum with the textbook recurrence in x (used by tests only, as an
    independent check away from x = 1)."""
    coef_l = np.asarray(coef_l, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    lmax = coef_l.shape[0] - 1
    c = (2.0 * np.arange(lmax + 1) + 1.0) * coef_l / (4.0 * np.pi)
    p_prev = np.ones_like(x)
    acc = c[0] * p_prev
    if lmax == 0:
        return acc
    p = x.copy()
    acc = acc + c[1] * p
    for l in range(1, lmax):
        p_next = ((2 * l + 1) * x * p - l * p_prev) / (l + 1)
        p_prev, p = p, p_next
        acc = acc + c[l + 1] * p
    return acc
