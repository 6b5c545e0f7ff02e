"""Oracle: the block-Jacobi factor of the system matrix of Section 4.2
(test infrastructure only; see package docstring).

Definitions followed
--------------------
* Section 4.2 rewrites the constrained-realisation system with the matrix
  D-hat + B-hat^T N^-1 B-hat (the operators of Eq. 16, the product of
  Eq. 15), and the paper's use of the local blocks is to build
  preconditioners or smoothers for iterative solvers of that system.  The
  simplest such preconditioner keeps the diagonal tile blocks: for every tile
  J, A_J = D_JJ + C_JJ, the stored blocks (J, J) of D-hat and of
  B-hat^T N^-1 B-hat.  The paper does not spell this step out; it is the
  consumer of its two operators that this library provides.
* A symmetric positive definite matrix A factors uniquely as A = U^T U with U
  upper triangular and a positive diagonal (Cholesky).  Written out row by row
  from the upper triangle of A:
      U_jj = sqrt(A_jj - sum_{c<j} U_cj^2),
      U_ji = (A_ji - sum_{c<j} U_cj U_ci) / U_jj        (i > j),
  so only the upper triangle of A is read.  The first j whose pivot
  A_jj - sum_{c<j} U_cj^2 is not positive reports info = j + 1 (the matrix is
  not positive definite); info = 0 means success.
* Applying the preconditioner to r solves A_J x_J = r_J for every tile:
  U^T y = r by forward substitution, then U x = y by back substitution.
"""
from __future__ import annotations

import numpy as np


def cholesky_upper(A):
    """(U, info): A = U^T U from the upper triangle of A (rows of U in order,
    each from the rows above it).  On failure U holds the rows completed so
    far and zeros below them."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    U = np.zeros((n, n))
    for j in range(n):
        pivot = A[j, j] - np.dot(U[:j, j], U[:j, j])
        if not pivot > 0.0:               # also NaN
            return U, j + 1
        U[j, j] = np.sqrt(pivot)
        U[j, j + 1:] = (A[j, j + 1:] - U[:j, j] @ U[:j, j + 1:]) / U[j, j]
    return U, 0


def diagonal_block_index(pairs, ntiles: int):
    """Position of the stored block (J, J) of every tile J in a stored-block
    list (J ascending, then K ascending; J is its own neighbour)."""
    idx = np.full(ntiles, -1, dtype=np.int64)
    for n, (J, K) in enumerate(pairs):
        if J == K:
            idx[J] = n
    assert (idx >= 0).all(), "every tile has its diagonal block"
    return idx


def factor_diag(D, C, pairs, ntiles: int, tiles=None):
    """U_J and info_J for A_J = D_JJ + C_JJ (C may be None: A_J = D_JJ).
    tiles: the tiles to factor (all by default).  Returns (U, info) with U of
    shape (len(tiles), k^2, k^2)."""
    idx = diagonal_block_index(pairs, ntiles)
    if tiles is None:
        tiles = range(ntiles)
    Us, infos = [], []
    for J in tiles:
        A = D[idx[J]] if C is None else D[idx[J]] + C[idx[J]]
        U, info = cholesky_upper(A)
        Us.append(U)
        infos.append(info)
    return np.stack(Us), np.array(infos, dtype=np.int32)


def solve_upper_factor(U, r):
    """x with (U^T U) x = r: forward substitution on U^T, then back
    substitution on U."""
    U = np.asarray(U, dtype=np.float64)
    n = U.shape[0]
    y = np.zeros(n)
    for i in range(n):                    # U^T y = r: row i of U^T is column i of U
        y[i] = (r[i] - np.dot(U[:i, i], y[:i])) / U[i, i]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):        # U x = y
        x[i] = (y[i] - np.dot(U[i, i + 1:], x[i + 1:])) / U[i, i]
    return x


def solve_diag(U, r, tiles=None):
    """Block-Jacobi application x_J = A_J^-1 r_J with A_J = U_J^T U_J, r and x
    in pixel order (tile J owns pixels [J k^2, (J+1) k^2)).  U: the factors of
    the tiles listed in tiles (all by default), in that order."""
    r = np.asarray(r, dtype=np.float64)
    k2 = U.shape[1]
    if tiles is None:
        tiles = range(U.shape[0])
    return np.stack([solve_upper_factor(U[n], r[J * k2:(J + 1) * k2]) for n, J in enumerate(tiles)])
