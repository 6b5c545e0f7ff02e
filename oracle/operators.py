"""Oracle: local blocks of D-hat and B-hat and the product B-hat^T N^-1 B-hat
(test infrastructure only; see package docstring).

Definitions followed
--------------------
* Eq. 16 with Y_2 = Y_1: D-hat = Y D Y^T and B-hat = Y B Y^T have elements
  d(n_i . n_j) and b(n_i . n_j) with the kernels of Eq. 10.
* Section 4.2: both are set to zero unless pixels i and j lie in the same or
  in neighbouring tiles.  B-hat is additionally cut at a radius R when one is
  given (gamma > R gives 0).
* Eq. 15: the operator needed is B-hat^T N^-1 B-hat with N^-1 diagonal in
  pixel space.  Its block between tiles J and K is
      C_JK = sum_{I in nbr(J) & nbr(K)} B_IJ^T diag(w_I) B_IK,
  because B-hat(p, q) vanishes unless tile(p) neighbours tile(q).  The stored
  blocks are the pairs (J, K) with K a neighbour of J and K >= J (the pattern
  of D-hat), each k^2 x k^2, rows and columns in tile-local order c*k + r.
* Section 4.1 (pixel-domain convolution): g_i = sum_j b(n_i . n_j) f_j, a plain
  sum over the samples j whose tile neighbours the tile of i (no quadrature
  weights), i.e. g = B-hat f; blockwise g_J = sum_{K in nbr(J)} B_JK f_K.
* Section 2.3 / 4.1: a block depends on the two tiles only through their
  bands and the exact rational phi offset between them, so blocks are cached
  on the key (band_I, band_J, (t_J T_I - t_I T_J) mod T_I T_J).  The brute
  force in ``oracle.brute`` checks this reuse against per-pair evaluation.

Pair geometry: with ring-local indices p, q on rings of n1, n2 pixels, the phi
difference is pi N / (n1 n2) with N = (2q+1) n1 - (2p+1) n2 reduced exactly into
(-n1 n2, n1 n2]; then y = 1 - cos(gamma) by the haversine formula
    y = 2 [ sin^2((theta1 - theta2)/2) + sin(theta1) sin(theta2) sin^2(dphi/2) ].
"""
from __future__ import annotations

import numpy as np

from .grid import Grid
from .kernel import legendre_series_in_y


def tile_pixel_geometry(g: Grid, tile: int):
    """For the k^2 pixels of a tile in local order a = c*k + r: ring index,
    ring-local pixel index, pixels on the ring, and the global pixel index."""
    k = g.k
    b = g.tile_band(tile)
    T = g.band_tiles[b]
    t = tile - g.band_tile0[b]
    c, r = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    c = c.ravel()
    r = r.ravel()
    ring = np.asarray(g.band_rings[b], dtype=np.int64)[r]
    pin = t * k + c
    nring = np.full(k * k, k * T, dtype=np.int64)
    gpix = g.band_pix0[b] + t * k * k + c * k + r
    return ring, pin.astype(np.int64), nring, gpix.astype(np.int64)


def pair_y(g: Grid, ring1, p1, n1, ring2, p2, n2):
    """y = 1 - cos(gamma) for pixel pairs given by (ring, ring-local index, ring
    length); all integer arrays broadcast together."""
    return pair_y_two(g, ring1, p1, n1, g, ring2, p2, n2)


def pair_y_two(g1: Grid, ring1, p1, n1, g2: Grid, ring2, p2, n2):
    """The same with the first pixel of each pair on grid g1 and the second on
    grid g2 (the rings' colatitudes come from each pixel's own grid)."""
    ring1, p1, n1, ring2, p2, n2 = np.broadcast_arrays(
        *(np.asarray(v, dtype=np.int64) for v in (ring1, p1, n1, ring2, p2, n2)))
    M = n1 * n2
    N = (2 * p2 + 1) * n1 - (2 * p1 + 1) * n2
    N = np.mod(N, 2 * M)
    N = np.where(N > M, N - 2 * M, N)
    dphi = np.pi * N.astype(np.float64) / M.astype(np.float64)
    th1 = g1.theta[ring1]
    th2 = g2.theta[ring2]
    s1 = g1.sin_theta[ring1]
    s2 = g2.sin_theta[ring2]
    return 2.0 * (np.sin(0.5 * (th1 - th2)) ** 2 + s1 * s2 * np.sin(0.5 * dphi) ** 2)


def block_y(g: Grid, I: int, J: int):
    """k^2 x k^2 matrix of y between the pixels of tile I (rows) and tile J (cols)."""
    r1, p1, n1, _ = tile_pixel_geometry(g, I)
    r2, p2, n2, _ = tile_pixel_geometry(g, J)
    return pair_y(g, r1[:, None], p1[:, None], n1[:, None], r2[None, :], p2[None, :], n2[None, :])


def unique_key(g: Grid, I: int, J: int):
    """(band_I, band_J, delta) with delta = (t_J T_I - t_I T_J) mod T_I T_J."""
    bI = g.tile_band(I)
    bJ = g.tile_band(J)
    TI, TJ = g.band_tiles[bI], g.band_tiles[bJ]
    tI, tJ = I - g.band_tile0[bI], J - g.band_tile0[bJ]
    return (bI, bJ, (tJ * TI - tI * TJ) % (TI * TJ))


def radius_to_y(radius):
    """y_R = 1 - cos(R) = 2 sin^2(R/2); None (no cut) for radius None or <= 0."""
    if radius is None or radius <= 0:
        return None
    return 2.0 * np.sin(0.5 * radius) ** 2


class LocalOperator:
    """The local part of a rotationally invariant operator with transfer
    function coef_l (b_l for B-hat, d_l for D-hat), blocks cached by the exact
    symmetry key."""

    def __init__(self, g: Grid, coef_l, radius=None):
        self.g = g
        self.coef = np.asarray(coef_l, dtype=np.float64)
        self.y_cut = radius_to_y(radius)
        self.cache = {}
        self._nbr = {}

    def neighbours(self, tile):
        if tile not in self._nbr:
            self._nbr[tile] = self.g.tile_neighbours(tile)
        return self._nbr[tile]

    def block(self, I: int, J: int):
        """B-hat restricted to rows in tile I and columns in tile J (zero block
        if the tiles are not neighbours)."""
        if J not in self.neighbours(I):
            k2 = self.g.k ** 2
            return np.zeros((k2, k2))
        key = unique_key(self.g, I, J)
        if key not in self.cache:
            y = block_y(self.g, I, J)
            val = legendre_series_in_y(self.coef, y)
            if self.y_cut is not None:
                val = np.where(y <= self.y_cut, val, 0.0)
            self.cache[key] = val
        return self.cache[key]


def stored_block_list(g: Grid):
    """Stored (J, K) pairs in output order: J ascending, then K ascending."""
    rp, col = g.stored_blocks()
    pairs = []
    for j in range(g.ntiles):
        for kk in col[rp[j]:rp[j + 1]]:
            pairs.append((j, int(kk)))
    return pairs


def two_hop_block_list(g: Grid):
    """Every block (J, K), K >= J, of B-hat^T N^-1 B-hat that can be nonzero
    when B-hat is local (Section 4.2): J and K have a common neighbour I
    (Eq. 15 sums over I in nbr(J) & nbr(K)).  Order: J ascending, then K."""
    nbr = [set(g.tile_neighbours(t)) for t in range(g.ntiles)]
    pairs = []
    for J in range(g.ntiles):
        ks = set()
        for I in nbr[J]:
            ks.update(K for K in nbr[I] if K >= J)
        pairs.extend((J, K) for K in sorted(ks))
    return pairs


def sample_D(g: Grid, d_l, radius=None, pairs=None):
    """All stored blocks D-hat_JK (Eq. 16, local truncation of Section 4.2)."""
    op = LocalOperator(g, d_l, radius)
    if pairs is None:
        pairs = stored_block_list(g)
    return np.stack([op.block(J, K) for J, K in pairs]) if pairs else np.zeros((0, g.k ** 2, g.k ** 2))


def btnb_block(op: LocalOperator, ninv, J: int, K: int):
    """C_JK = sum_{I in nbr(J) & nbr(K)} B_IJ^T diag(w_I) B_IK   (Eq. 15)."""
    g = op.g
    k2 = g.k ** 2
    acc = np.zeros((k2, k2))
    common = sorted(set(op.neighbours(J)) & set(op.neighbours(K)))
    for I in common:
        w = ninv[I * k2:(I + 1) * k2]       # tile I's pixels are contiguous, local order
        acc += op.block(I, J).T @ (w[:, None] * op.block(I, K))
    return acc


def sample_BtNB(g: Grid, b_l, ninv, radius=None, pairs=None):
    """All stored blocks of B-hat^T N^-1 B-hat (Eq. 15) with N^-1 = diag(ninv),
    ninv in pixel order."""
    ninv = np.asarray(ninv, dtype=np.float64)
    op = LocalOperator(g, b_l, radius)
    if pairs is None:
        pairs = stored_block_list(g)
    if not pairs:
        return np.zeros((0, g.k ** 2, g.k ** 2))
    return np.stack([btnb_block(op, ninv, J, K) for J, K in pairs])


def convolve(g: Grid, b_l, f, radius=None, tiles=None):
    """Pixel-domain convolution of Section 4.1, g = B-hat f: for every output
    tile J, g_J = sum_{K in nbr(J)} B_JK f_K with the local blocks above (f and
    g in pixel order).  tiles: the output tiles to compute (all by default);
    returns an array (len(tiles), k^2)."""
    f = np.asarray(f, dtype=np.float64)
    op = LocalOperator(g, b_l, radius)
    k2 = g.k ** 2
    if tiles is None:
        tiles = range(g.ntiles)
    out = []
    for J in tiles:
        acc = np.zeros(k2)
        for K in op.neighbours(J):
            acc += op.block(J, K) @ f[K * k2:(K + 1) * k2]
        out.append(acc)
    return np.stack(out) if out else np.zeros((0, k2))

