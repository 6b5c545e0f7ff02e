"""Oracle: spherical harmonic transforms on the SymPix geometry and the N^-1
degrade of Eq. 14 (test infrastructure only: only tests/, the smoke check and
the CPU baseline of bench.py use it).

Conventions.  Real orthonormal spherical harmonics without the Condon-Shortley
phase, so that the operator Y of Eqs. 12-16 is a real matrix and Y^T is its
plain transpose:

    Y_{l,0}  = lambda_l0(theta)
    Y_{l,m}  = sqrt(2) lambda_lm(theta) cos(m phi)      (m > 0)
    Y_{l,-m} = sqrt(2) lambda_lm(theta) sin(m phi)      (m > 0)

with lambda_lm(theta) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta) and
P_l^m >= 0 near the north pole.  A coefficient vector of band limit L has
(L+1)^2 entries, entry l^2 + l + m holding the coefficient of Y_{l,m}.

    synthesis   f = Y a                      (Eq. 1 read right to left)
    adjoint     a = Y^T f                    (no quadrature weights)
    analysis    a = Y^T W f                  (the quadrature rule of Eq. 1)
    degrade     theta_2 = W_2 Y_2 Y_obs^T theta    (Eq. 14)

W is diagonal with, for a pixel on ring r holding n_r pixels, the weight
w_r^GL * 2 pi / n_r (the Gauss-Legendre weight of the ring, Section 2.1, times
the equal spacing in phi).  The transforms are plain sums over every pixel and
every mode; no mode is dropped near the poles (the cut of Eq. 2 is what makes
SymPix rings shorter than 2 L + 1 there, so analysis of synthesis is not the
identity on those grids: Table 1's error columns).

lambda_lm is computed by the textbook recurrences, started from lambda_mm =
sqrt((2m+1)/(4 pi) (2m)!) / (2^m m!) sin^m(theta) and carried with power-of-two
rescaling, so that values far below the double range (near the poles at high
m) do not stop the recurrence from reaching the values that matter.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid

_RESCALE = 2.0 ** 300


def lambda_table(lmax: int, theta) -> np.ndarray:
    """lambda_lm(theta) for 0 <= m <= l <= lmax: array [lmax+1 (l), lmax+1 (m), ntheta],
    zero for m > l."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    x = np.cos(theta)
    s = np.sin(theta)
    out = np.zeros((lmax + 1, lmax + 1, theta.size))
    # lambda_mm as mant * 2^e2, built by the product recurrence in m
    mant = np.full(theta.size, np.sqrt(1.0 / (4.0 * np.pi)))
    e2 = np.zeros(theta.size, dtype=np.int64)
    for m in range(lmax + 1):
        if m > 0:
            mant = mant * np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s
            small = np.abs(mant) < 1.0 / _RESCALE
            mant = np.where(small, mant * _RESCALE, mant)
            e2 = np.where(small, e2 - 300, e2)
        # l recurrence for this m, on values scaled by 2^-e (e per theta)
        p_prev = np.zeros(theta.size)          # lambda_{l-2, m}
        p = mant.copy()                        # lambda_{l-1, m} at l = m + 1
        e = e2.copy()
        out[m, m] = np.ldexp(p, e)
        for l in range(m + 1, lmax + 1):
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            if l == m + 1:
                q = a * x * p
            else:
                b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                q = a * (x * p - b * p_prev)
            big = np.abs(q) > _RESCALE
            q = np.where(big, q / _RESCALE, q)
            p = np.where(big, p / _RESCALE, p)
            e = np.where(big, e + 300, e)
            p_prev, p = p, q
            out[l, m] = np.ldexp(p, e)
    return out


def lambda_m(lmax: int, m: int, theta) -> np.ndarray:
    """lambda_lm(theta) of one order m for l = m .. lmax: array [lmax+1-m, ntheta].
    The same steps as lambda_table (the product recurrence in m up to m, then
    the recurrence in l), for checks at band limits where the full table is
    too large."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    x = np.cos(theta)
    s = np.sin(theta)
    mant = np.full(theta.size, np.sqrt(1.0 / (4.0 * np.pi)))
    e2 = np.zeros(theta.size, dtype=np.int64)
    for k in range(1, m + 1):
        mant = mant * np.sqrt((2.0 * k + 1.0) / (2.0 * k)) * s
        small = np.abs(mant) < 1.0 / _RESCALE
        mant = np.where(small, mant * _RESCALE, mant)
        e2 = np.where(small, e2 - 300, e2)
    out = np.zeros((lmax + 1 - m, theta.size))
    p_prev = np.zeros(theta.size)
    p = mant.copy()
    e = e2.copy()
    out[0] = np.ldexp(p, e)
    for l in range(m + 1, lmax + 1):
        a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        if l == m + 1:
            q = a * x * p
        else:
            b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            q = a * (x * p - b * p_prev)
        big = np.abs(q) > _RESCALE
        q = np.where(big, q / _RESCALE, q)
        p = np.where(big, p / _RESCALE, p)
        e = np.where(big, e + 300, e)
        p_prev, p = p, q
        out[l - m] = np.ldexp(p, e)
    return out


def _index(l: int, m: int) -> int:
    return l * l + l + m


def _ring_tables(g: Grid):
    ring, pin, nr, phi = g.pixel_coords()
    return ring, phi


def synthesis(g: Grid, a, lmax: int, rings=None) -> np.ndarray:
    """f = Y a on every pixel of g (Eq. 1 as a sum over modes); with rings
    (a list of ring indices), f on the pixels of those rings only, in pixel
    order (the same sums, so the same values)."""
    a = np.asarray(a, dtype=np.float64)
    if a.shape != ((lmax + 1) ** 2,):
        raise ValueError("a must have (lmax+1)^2 entries")
    ring, phi = _ring_tables(g)
    if rings is None:
        lam = lambda_table(lmax, g.theta)                   # [l, m, ring]
    else:
        rings = list(rings)
        keep = np.isin(ring, rings)
        ring = np.searchsorted(np.asarray(sorted(rings)), ring[keep])   # position among the chosen rings
        phi = phi[keep]
        lam = lambda_table(lmax, np.asarray(g.theta)[sorted(rings)])
    ls = np.arange(lmax + 1)
    f = np.zeros(len(ring))
    for m in range(lmax + 1):
        l_m = ls[m:]
        cm = a[l_m * l_m + l_m + m]
        Fc = np.einsum("l,lr->r", cm, lam[m:, m, :])         # per ring
        if m == 0:
            f += Fc[ring]
            continue
        sm = a[l_m * l_m + l_m - m]
        Fs = np.einsum("l,lr->r", sm, lam[m:, m, :])
        f += np.sqrt(2.0) * (Fc[ring] * np.cos(m * phi) + Fs[ring] * np.sin(m * phi))
    return f


def adjoint(g: Grid, f, lmax: int) -> np.ndarray:
    """a = Y^T f: the transpose of synthesis (no quadrature weights)."""
    f = np.asarray(f, dtype=np.float64)
    if f.shape != (g.npix,):
        raise ValueError("f must have npix entries")
    ring, phi = _ring_tables(g)
    lam = lambda_table(lmax, g.theta)
    a = np.zeros((lmax + 1) ** 2)
    for m in range(lmax + 1):
        if m == 0:
            Gc = np.bincount(ring, weights=f, minlength=g.nrings)
        else:
            Gc = np.sqrt(2.0) * np.bincount(ring, weights=f * np.cos(m * phi), minlength=g.nrings)
            Gs = np.sqrt(2.0) * np.bincount(ring, weights=f * np.sin(m * phi), minlength=g.nrings)
        for l in range(m, lmax + 1):
            a[_index(l, m)] = lam[l, m, :] @ Gc
            if m > 0:
                a[_index(l, -m)] = lam[l, m, :] @ Gs
    return a


def pixel_weights(g: Grid) -> np.ndarray:
    """Diagonal of W: Gauss-Legendre ring weight times 2 pi / n_ring per pixel."""
    ring, pin, nr, phi = g.pixel_coords()
    return g.weight[ring] * 2.0 * np.pi / nr


def analysis(g: Grid, f, lmax: int) -> np.ndarray:
    """a = Y^T W f (the quadrature rule of Eq. 1)."""
    return adjoint(g, np.asarray(f, dtype=np.float64) * pixel_weights(g), lmax)


def degrade(g_obs: Grid, g2: Grid, theta_obs, lmax: int) -> np.ndarray:
    """theta_2 = W_2 Y_2 Y_obs^T theta (Eq. 14): Y_obs^T without ring weights,
    then synthesis on the target grid and its quadrature weights."""
    return pixel_weights(g2) * synthesis(g2, adjoint(g_obs, theta_obs, lmax), lmax)
