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
