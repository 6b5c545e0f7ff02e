"""Oracle: B-hat between two SymPix grids (test infrastructure only; see the
package docstring).

Definitions followed
--------------------
* Eq. 13 moves N^-1 onto an auxiliary SymPix grid Y_2, which need not be the
  grid Y_1 of the unknowns; Eq. 16 then defines B-hat = Y_2 B Y_1^T, a matrix
  with a row per pixel of Y_2 and a column per pixel of Y_1.  Its element
  (i, j) is b(n_i . n_j) with the kernel of Eq. 10 summed over the multipoles
  both transforms carry, l <= min(lmax_1, lmax_2) (Y_1^T and Y_2 pass no
  others, and B is diagonal in l).
* Section 4.2 keeps an element only when the tiles of its two sample points
  are the same or neighbours; B-hat is additionally cut at a radius R when one
  is given.
* Eq. 15: the operator needed is B-hat^T N_2^-1 B-hat with N_2^-1 diagonal on
  the pixels of Y_2.  Its block between tiles J and K of Y_1 is
      C_JK = sum_{I in nbr(J) & nbr(K)} B_IJ^T diag(w_I) B_IK
  over the tiles I of Y_2 neighbouring both, a k_1^2 x k_1^2 block; B_IJ is
  k_2^2 x k_1^2 (rectangular when the grids' tile sizes differ).

Reading (the paper does not say when a tile of Y_2 and a tile of Y_1 are
"neighbouring"): every tile covers a closed rectangle in (theta, phi), and two
tiles of the two grids are neighbours when their rectangles meet (touching
counts).  A tile's phi range is [t/T, (t+1)/T] of a turn; its band's
colatitude range is [i k/R, (i+1) k/R] pi for north band i of a grid with R
rings (the mirror image for south band i).  The j-th Gauss-Legendre ring lies
strictly inside [j/R, (j+1)/R] pi (the zeros of P_R obey
(j + 1/2)/(R + 1/2) < theta_j / pi < (j + 1)/(R + 1/2)), so each band's rings
lie inside its range.  On one grid, bands that follow each other share an edge
(the two equatorial bands meet at pi/2) and no others meet, so with Y_2 = Y_1
the relation is the single-grid one (same band t-1, t, t+1; neighbouring bands
by closed phi intervals): the two-grid operator then equals the one-grid
operator exactly.  Everything is compared in integers (rational range ends).
"""
from __future__ import annotations

import numpy as np

from .grid import Grid
from .kernel import legendre_series_in_y
from .operators import pair_y_two, radius_to_y, tile_pixel_geometry


def band_colatitude(g: Grid, b: int):
    """Colatitude range of storage band b as (lo, hi, den): [lo/den, hi/den] pi."""
    i, south = divmod(b, 2)
    R, k = g.nrings, g.k
    if south:
        return (R - (i + 1) * k, R - i * k, R)
    return (i * k, (i + 1) * k, R)


def ranges_meet(e1, e2) -> bool:
    """Closed rational ranges [a1/d1, b1/d1] and [a2/d2, b2/d2] meet."""
    a1, b1, d1 = e1
    a2, b2, d2 = e2
    return a1 * d2 <= b2 * d1 and a2 * d1 <= b1 * d2


def phi_meet(t1: int, T1: int, t2: int, T2: int) -> bool:
    """Closed phi intervals [t1/T1, (t1+1)/T1] and [t2/T2, (t2+1)/T2] meet
    modulo one turn (integers after scaling by T1 T2)."""
    M = T1 * T2
    lo1, hi1 = t1 * T2, (t1 + 1) * T2
    lo2, hi2 = t2 * T1, (t2 + 1) * T1
    return any(lo1 <= hi2 + s and lo2 + s <= hi1 for s in (-M, 0, M))


def cross_neighbours(g2: Grid, g1: Grid, J: int):
    """Sorted tiles of g2 whose rectangle meets that of tile J of g1."""
    bJ = g1.tile_band(J)
    eJ = band_colatitude(g1, bJ)
    TJ = g1.band_tiles[bJ]
    tJ = J - g1.band_tile0[bJ]
    out = []
    for b2 in range(len(g2.band_tiles)):
        if not ranges_meet(band_colatitude(g2, b2), eJ):
            continue
        T2 = g2.band_tiles[b2]
        for t2 in range(T2):
            if phi_meet(t2, T2, tJ, TJ):
                out.append(g2.band_tile0[b2] + t2)
    return sorted(out)


def cross_adjacency(g2: Grid, g1: Grid):
    """The relation as CSR over the tiles I of g2: for each, the tiles J of g1
    it neighbours (ascending)."""
    rows = [[] for _ in range(g2.ntiles)]
    for J in range(g1.ntiles):
        for I in cross_neighbours(g2, g1, J):
            rows[I].append(J)
    rp = np.zeros(g2.ntiles + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.fromiter((c for r in rows for c in r), dtype=np.int32, count=int(rp[-1]))
    return rp, col


def cross_key(g2: Grid, I: int, g1: Grid, J: int):
    """(band of I in g2, band of J in g1, delta = (t_J T_I - t_I T_J) mod T_I T_J):
    the block depends on the pair only through this key (Section 2.3: a joint
    rotation by a multiple of 2 pi / gcd(T_I, T_J) maps the two bands' pixels
    onto themselves)."""
    bI = g2.tile_band(I)
    bJ = g1.tile_band(J)
    TI, TJ = g2.band_tiles[bI], g1.band_tiles[bJ]
    tI, tJ = I - g2.band_tile0[bI], J - g1.band_tile0[bJ]
    return (bI, bJ, (tJ * TI - tI * TJ) % (TI * TJ))


def effective_lmax(g2: Grid, g1: Grid) -> int:
    return min(g1.lmax, g2.lmax)


class CrossOperator:
    """The local part of B-hat = Y_2 B Y_1^T with transfer function coef_l,
    blocks cached by the exact key."""

    def __init__(self, g2: Grid, g1: Grid, coef_l, radius=None):
        self.g2, self.g1 = g2, g1
        L = effective_lmax(g2, g1)
        coef = np.zeros(L + 1)
        c = np.asarray(coef_l, dtype=np.float64)[:L + 1]
        coef[:c.size] = c
        self.coef = coef
        self.y_cut = radius_to_y(radius)
        self.cache = {}
        self._nbr = {}

    def neighbours(self, J: int):
        """Tiles of Y_2 neighbouring tile J of Y_1."""
        if J not in self._nbr:
            self._nbr[J] = cross_neighbours(self.g2, self.g1, J)
        return self._nbr[J]

    def block(self, I: int, J: int):
        """B-hat restricted to rows in tile I of Y_2 and columns in tile J of
        Y_1 (k_2^2 x k_1^2; zero if the tiles are not neighbours)."""
        if I not in self.neighbours(J):
            return np.zeros((self.g2.k ** 2, self.g1.k ** 2))
        key = cross_key(self.g2, I, self.g1, J)
        if key not in self.cache:
            r2, p2, n2, _ = tile_pixel_geometry(self.g2, I)
            r1, p1, n1, _ = tile_pixel_geometry(self.g1, J)
            y = pair_y_two(self.g2, r2[:, None], p2[:, None], n2[:, None], self.g1, r1[None, :], p1[None, :],
                           n1[None, :])
            val = legendre_series_in_y(self.coef, y)
            if self.y_cut is not None:
                val = np.where(y <= self.y_cut, val, 0.0)
            self.cache[key] = val
        return self.cache[key]


def btnb_cross_block(op: CrossOperator, ninv2, J: int, K: int):
    """C_JK = sum_{I in nbr(J) & nbr(K)} B_IJ^T diag(w_I) B_IK  (Eq. 15), I over
    the tiles of Y_2, w = N_2^-1 in the pixel order of Y_2."""
    k2 = op.g2.k ** 2
    acc = np.zeros((op.g1.k ** 2, op.g1.k ** 2))
    common = sorted(set(op.neighbours(J)) & set(op.neighbours(K)))
    for I in common:
        w = ninv2[I * k2:(I + 1) * k2]
        acc += op.block(I, J).T @ (w[:, None] * op.block(I, K))
    return acc


def sample_BtNB_cross(g2: Grid, g1: Grid, b_l, ninv2, radius=None, pairs=None):
    """Stored blocks (J, K) of Y_1 (the pattern of D-hat: K a neighbour of J,
    K >= J) of B-hat^T N_2^-1 B-hat."""
    from .operators import stored_block_list
    ninv2 = np.asarray(ninv2, dtype=np.float64)
    op = CrossOperator(g2, g1, b_l, radius)
    if pairs is None:
        pairs = stored_block_list(g1)
    if not pairs:
        return np.zeros((0, g1.k ** 2, g1.k ** 2))
    return np.stack([btnb_cross_block(op, ninv2, J, K) for J, K in pairs])


def sample_B_cross(g2: Grid, g1: Grid, b_l, radius=None):
    """Every nonzero block (I, J) of B-hat in the order of cross_adjacency
    (I of Y_2 ascending, then J of Y_1 ascending)."""
    op = CrossOperator(g2, g1, b_l, radius)
    rp, col = cross_adjacency(g2, g1)
    blocks = [op.block(I, int(J)) for I in range(g2.ntiles) for J in col[rp[I]:rp[I + 1]]]
    return np.stack(blocks) if blocks else np.zeros((0, g2.k ** 2, g1.k ** 2))
