"""Pins for the block-Jacobi factor oracle (Section 4.2's system matrix,
Cholesky of its diagonal tile blocks): an exact integer example, uniqueness
of the factor, an independent library factorisation, the upper-triangle-only
contract, failure reporting, and the solve against the matrix it inverts."""
import numpy as np
import pytest
import scipy.linalg

from oracle import grid as G
from oracle import operators as O
from oracle import precond as P
from workloads import synth as S


def _spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def test_exact_integer_example():
    # A = U^T U with U = [[2, 6, -8], [0, 1, 5], [0, 0, 3]]: every step is exact in FP64
    A = np.array([[4.0, 12.0, -16.0], [12.0, 37.0, -43.0], [-16.0, -43.0, 98.0]])
    U, info = P.cholesky_upper(A)
    assert info == 0
    assert np.array_equal(U, np.array([[2.0, 6.0, -8.0], [0.0, 1.0, 5.0], [0.0, 0.0, 3.0]]))


@pytest.mark.parametrize("n,seed", [(5, 1), (64, 2)])
def test_factor_is_the_unique_one(n, seed):
    rng = np.random.default_rng(seed)
    U0 = np.triu(rng.uniform(-1.0, 1.0, (n, n)), 1) + np.diag(rng.uniform(2.0, 3.0, n))
    U, info = P.cholesky_upper(U0.T @ U0)
    assert info == 0
    assert np.abs(U - U0).max() <= 1e-12 * np.abs(U0).max()


def test_matches_an_independent_factorisation():
    A = _spd(64, 3)
    U, info = P.cholesky_upper(A)
    assert info == 0
    ref = scipy.linalg.cholesky(A, lower=False)
    assert np.abs(U - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(U.T @ U - A).max() <= 1e-13 * np.abs(A).max()


def test_reads_only_the_upper_triangle():
    A = _spd(16, 4)
    B = A.copy()
    B[np.tril_indices(16, -1)] = np.nan
    Ua, _ = P.cholesky_upper(A)
    Ub, info = P.cholesky_upper(B)
    assert info == 0 and np.array_equal(Ua, Ub)


@pytest.mark.parametrize("A,info", [
    (np.diag([1.0, -1.0, 1.0]), 2),
    (np.array([[1.0, 2.0], [2.0, 1.0]]), 2),      # second pivot 1 - 4 = -3
    (np.zeros((3, 3)), 1),
    (np.array([[4.0, 2.0], [2.0, 1.0]]), 2),      # singular: second pivot exactly 0
    (np.array([[np.nan, 0.0], [0.0, 1.0]]), 1),
])
def test_reports_the_first_failing_pivot(A, info):
    assert P.cholesky_upper(A)[1] == info


def test_solve_inverts_the_matrix():
    A = _spd(64, 5, cond=1e4)
    U, _ = P.cholesky_upper(A)
    r = np.random.default_rng(6).standard_normal(64)
    x = P.solve_upper_factor(U, r)
    assert np.abs(A @ x - r).max() <= 1e-11 * np.abs(r).max()
    # a diagonal matrix: x = r / a exactly (U = sqrt(a), two divisions by it)
    a = np.array([4.0, 9.0, 16.0, 0.25])
    Ud, _ = P.cholesky_upper(np.diag(a))
    assert np.array_equal(P.solve_upper_factor(Ud, np.array([8.0, 27.0, 32.0, 1.0])), np.array([2.0, 3.0, 2.0, 4.0]))


@pytest.mark.parametrize("lmax,k,margin", [(16, 2, 0.0), (20, 2, 0.0), (24, 4, None)])
def test_sympix_diagonal_blocks_are_positive_definite_and_reconstruct(lmax, k, margin):
    """A_J = D_JJ + C_JJ of the synthetic workload recipe: every tile factors,
    U_J^T U_J gives A_J back, and the solve inverts A_J."""
    g = G.make_grid(lmax, k, polar_margin=margin)
    rng = np.random.default_rng(11)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    pairs = O.stored_block_list(g)
    D = O.sample_D(g, S.prior(lmax), None, pairs)
    C = O.sample_BtNB(g, b_l, ninv, R, pairs)
    idx = P.diagonal_block_index(pairs, g.ntiles)
    assert all(pairs[idx[J]] == (J, J) for J in range(g.ntiles))
    U, info = P.factor_diag(D, C, pairs, g.ntiles)
    assert (info == 0).all()
    for J in range(g.ntiles):
        A = D[idx[J]] + C[idx[J]]
        assert np.abs(U[J].T @ U[J] - A).max() <= 1e-13 * np.abs(A).max()
        assert np.array_equal(U[J], np.triu(U[J]))
    r = rng.standard_normal(g.npix)
    x = P.solve_diag(U, r)
    k2 = k * k
    for J in range(g.ntiles):
        A = D[idx[J]] + C[idx[J]]
        assert np.abs(A @ x[J] - r[J * k2:(J + 1) * k2]).max() <= 1e-9 * np.abs(r).max() * np.linalg.cond(A) * 1e-3
    # D-hat alone factors too (C = None)
    _, info_d = P.factor_diag(D, None, pairs, g.ntiles)
    assert (info_d == 0).all()
