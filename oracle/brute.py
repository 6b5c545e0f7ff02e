"""Oracle brute force (test infrastructure only; see package docstring).

Builds the local operator of Section 4.2 pair by pair, with no symmetry keys
and no block cache, and forms B-hat^T N^-1 B-hat with a sparse product.  The
geometry comes from 3-D unit vectors (|n1 - n2|^2 = 2 (1 - cos gamma)) rather
than from the haversine form used by ``oracle.operators``, so the two paths
share no geometry code; the tile pattern is checked separately.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .grid import Grid
from .kernel import legendre_series_in_y


def unit_vectors(g: Grid):
    ring, pin, nr, phi = g.pixel_coords()
    th = g.theta[ring]
    st = np.sin(th)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(th)], axis=1)


def pattern_pairs(g: Grid):
    """All (i, j) pixel pairs whose tiles neighbour each other (ordered pairs)."""
    k2 = g.k ** 2
    rp, col = g.adjacency()
    rows = []
    cols = []
    loc = np.arange(k2)
    for I in range(g.ntiles):
        for J in col[rp[I]:rp[I + 1]]:
            ii, jj = np.meshgrid(I * k2 + loc, int(J) * k2 + loc, indexing="ij")
            rows.append(ii.ravel())
            cols.append(jj.ravel())
    return np.concatenate(rows), np.concatenate(cols)


def local_operator_sparse(g: Grid, coef_l, radius=None):
    """Sparse Npix x Npix local operator, every element evaluated directly."""
    v = unit_vectors(g)
    i, j = pattern_pairs(g)
    diff = v[i] - v[j]
    y = 0.5 * np.einsum("ij,ij->i", diff, diff)
    val = legendre_series_in_y(coef_l, y)
    if radius is not None and radius > 0:
        val = np.where(y <= 2.0 * np.sin(0.5 * radius) ** 2, val, 0.0)
    return sp.csr_matrix((val, (i, j)), shape=(g.npix, g.npix))


def btnb_sparse(g: Grid, b_l, ninv, radius=None):
    """B-hat^T diag(ninv) B-hat over the whole grid (all hops)."""
    B = local_operator_sparse(g, b_l, radius)
    W = sp.diags(np.asarray(ninv, dtype=np.float64))
    return (B.T @ W @ B).tocsr()


def extract_blocks(M, g: Grid, pairs):
    """Dense k^2 x k^2 blocks (J, K) of a sparse pixel-space matrix."""
    k2 = g.k ** 2
    out = np.zeros((len(pairs), k2, k2))
    for n, (J, K) in enumerate(pairs):
        out[n] = M[J * k2:(J + 1) * k2, K * k2:(K + 1) * k2].toarray()
    return out


# ---------------------------------------------------------------------------
# Two grids (Eqs. 13 and 16): B-hat = Y_2 B Y_1^T element by element
# ---------------------------------------------------------------------------

def tile_centres(g: Grid):
    """Per tile, its centre as (colatitude / pi, longitude / turn) in floating
    point: the middle of its band's range [i k/R, (i+1) k/R] (mirrored in the
    south) and of [t/T, (t+1)/T]."""
    out = np.zeros((g.ntiles, 2))
    k, R = g.k, g.nrings
    for b in range(len(g.band_tiles)):
        i, south = divmod(b, 2)
        lo, hi = (i * k, (i + 1) * k) if not south else (R - (i + 1) * k, R - i * k)
        T = g.band_tiles[b]
        for t in range(T):
            out[g.band_tile0[b] + t] = ((lo + hi) / (2 * R), (2 * t + 1) / (2 * T))
    return out


def cross_relation_dense(g2: Grid, g1: Grid):
    """Boolean ntiles_2 x ntiles_1 matrix of the two-grid tile relation, built
    in floating point: each tile centre of g2 located in g1 by sorted band
    edges and a floor, then the one-grid neighbours of the tile found."""
    k, R = g1.k, g1.nrings
    # band edges of g1 from the north pole, with the storage band of each interval
    edges, bands = [], []
    for i in range(g1.nbands_hemi):
        edges.append(i * k / R)
        bands.append(2 * i)
    for i in reversed(range(g1.nbands_hemi)):
        edges.append((R - (i + 1) * k) / R)
        bands.append(2 * i + 1)
    edges = np.array(edges)
    rel = np.zeros((g2.ntiles, g1.ntiles), dtype=bool)
    for I, (th, ph) in enumerate(tile_centres(g2)):
        b = bands[int(np.searchsorted(edges, th, side="right")) - 1]
        T = g1.band_tiles[b]
        J0 = g1.band_tile0[b] + int(np.floor(ph * T))
        rel[I, g1.tile_neighbours(J0)] = True
    return rel


def cross_operator_dense(g2: Grid, g1: Grid, coef_l, radius=None):
    """Dense Npix_2 x Npix_1 B-hat: every element evaluated directly from 3-D
    unit vectors, kept where the two pixels' tiles are related (and within
    radius); the kernel sums l <= min(lmax_1, lmax_2)."""
    L = min(g1.lmax, g2.lmax)
    coef = np.zeros(L + 1)
    c = np.asarray(coef_l, dtype=np.float64)[:L + 1]
    coef[:c.size] = c
    v2, v1 = unit_vectors(g2), unit_vectors(g1)
    diff = v2[:, None, :] - v1[None, :, :]
    y = 0.5 * np.einsum("ijk,ijk->ij", diff, diff)
    val = legendre_series_in_y(coef, y.ravel()).reshape(y.shape)
    rel = cross_relation_dense(g2, g1)
    keep = np.repeat(np.repeat(rel, g2.k ** 2, axis=0), g1.k ** 2, axis=1)
    if radius is not None and radius > 0:
        keep &= y <= 2.0 * np.sin(0.5 * radius) ** 2
    return np.where(keep, val, 0.0)
