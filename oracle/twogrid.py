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
"neighbouring"): the tile organisation that truncates is that of Y_1, the grid
of the unknowns.  A tile of Y_2 is placed in the tile of Y_1 that contains its
centre, and tile I of Y_2 neighbours tile J of Y_1 when that tile is J or one
of J's neighbours (the one-grid relation of Section 2.2).  The truncation then
reaches as far from J as it does on one grid, whatever the resolution of Y_2.
Centres and ranges are exact rationals: band i of a grid with R rings spans
the colatitudes [i k/R, (i+1) k/R] pi in the north (the mirror image in the
south) and tile t of a band of T tiles the longitudes [t/T, (t+1)/T] of a turn;
a tile's centre is the middle of both.  The j-th Gauss-Legendre ring lies
strictly inside [j/R, (j+1)/R] pi (the zeros of P_R obey
(j + 1/2)/(R + 1/2) < theta_j / pi < (j + 1)/(R + 1/2)), so each band's rings
lie inside its range.  A centre on a boundary of Y_1 belongs to the band or
tile on its south or east side (half-open ranges).  With Y_2 = Y_1 every tile
contains its own centre and the relation is the one-grid one, so the two-grid
operator then equals the one-grid operator exactly.  Which pairs are kept does
not change any block's values: a kept block depends only on the two bands and
the exact phi offset between the tiles, as on one grid.
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


def containing_tile(g1: Grid, th_num: int, th_den: int, ph_num: int, ph_den: int) -> int:
    """The tile of g1 containing the point of colatitude (th_num/th_den) pi and
    longitude ph_num/ph_den of a turn (half-open ranges, exact integers)."""
    for b in range(len(g1.band_tiles)):
        lo, hi, den = band_colatitude(g1, b)
        if lo * th_den <= th_num * den < hi * th_den:
            T = g1.band_tiles[b]
            return g1.band_tile0[b] + (ph_num * T) // ph_den
    raise ValueError("colatitude outside [0, pi)")


def tile_centre_container(g2: Grid, g1: Grid, I: int) -> int:
    """The tile of g1 that contains the centre of tile I of g2."""
    b = g2.tile_band(I)
    lo, hi, den = band_colatitude(g2, b)
    T = g2.band_tiles[b]
    t = I - g2.band_tile0[b]
    return containing_tile(g1, lo + hi, 2 * den, 2 * t + 1, 2 * T)


def centre_containers(g2: Grid, g1: Grid):
    """containing_tile for the centre of every tile of g2 at once (the same
    half-open tests, over the bands of g1 in turn)."""
    lo2 = np.zeros(g2.ntiles, dtype=np.int64)
    den2 = np.zeros(g2.ntiles, dtype=np.int64)
    ph_num = np.zeros(g2.ntiles, dtype=np.int64)
    ph_den = np.zeros(g2.ntiles, dtype=np.int64)
    for b in range(len(g2.band_tiles)):
        lo, hi, den = band_colatitude(g2, b)
        T = g2.band_tiles[b]
        sl = slice(g2.band_tile0[b], g2.band_tile0[b] + T)
        lo2[sl], den2[sl] = lo + hi, 2 * den
        ph_num[sl], ph_den[sl] = 2 * np.arange(T) + 1, 2 * T
    out = np.full(g2.ntiles, -1, dtype=np.int64)
    for b in range(len(g1.band_tiles)):
        lo, hi, den = band_colatitude(g1, b)
        inside = (lo * den2 <= lo2 * den) & (lo2 * den < hi * den2)
        T = g1.band_tiles[b]
        out[inside] = g1.band_tile0[b] + (ph_num[inside] * T) // ph_den[inside]
    assert (out >= 0).all()
    return out


def cross_adjacency(g2: Grid, g1: Grid):
    """The relation as CSR over the tiles I of g2: the tiles J of g1 it
    neighbours, ascending (the neighbours of the tile of g1 holding I's
    centre, itself included)."""
    rows = [g1.tile_neighbours(tile_centre_container(g2, g1, I)) for I in range(g2.ntiles)]
    rp = np.zeros(g2.ntiles + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.fromiter((c for r in rows for c in r), dtype=np.int32, count=int(rp[-1]))
    return rp, col


def cross_neighbours(g2: Grid, g1: Grid, J: int):
    """Sorted tiles of g2 neighbouring tile J of g1."""
    nj = set(g1.tile_neighbours(J))
    return [I for I in range(g2.ntiles) if tile_centre_container(g2, g1, I) in nj]


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
        self._container = None

    def neighbours(self, J: int):
        """Tiles of Y_2 neighbouring tile J of Y_1."""
        if J not in self._nbr:
            if self._container is None:
                self._container = centre_containers(self.g2, self.g1)
            nj = np.array(self.g1.tile_neighbours(J))
            self._nbr[J] = [int(I) for I in np.flatnonzero(np.isin(self._container, nj))]
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
