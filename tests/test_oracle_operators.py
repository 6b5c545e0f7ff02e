"""Pins for the oracle's local operators and B-hat^T N^-1 B-hat (Eqs. 15-16,
Section 4.2): brute force without symmetry reuse, closed forms (delta map,
linearity) and the grid's symmetries."""
import numpy as np
import pytest

from oracle import brute as BR
from oracle import grid as G
from oracle import operators as O
from workloads import synth as S

# small grids whose bands change tile count by three different ratios
TRANSITION_GRIDS = [(20, 2, 0.0), (32, 2, 0.0), (34, 2, 2.0)]


def _inputs(g, seed=7):
    rng = np.random.default_rng(seed)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    b_l, R = S.gaussian_beam(g.lmax, g.npix, 3.0)
    return ninv, b_l, R


def _gate(C, ref, pairs):
    """max |C - ref| / M_J with M_J the largest |ref| in block-row J."""
    rowmax = {}
    for n, (J, K) in enumerate(pairs):
        rowmax[J] = max(rowmax.get(J, 0.0), np.abs(ref[n]).max())
    return max(np.abs(C[n] - ref[n]).max() / rowmax[J] for n, (J, K) in enumerate(pairs))


@pytest.mark.parametrize("lmax,k,margin", TRANSITION_GRIDS)
def test_btnb_and_D_match_dense_brute_force(lmax, k, margin):
    g = G.make_grid(lmax, k, polar_margin=margin)
    ninv, b_l, R = _inputs(g)
    d_l = S.prior(lmax)
    pairs = O.stored_block_list(g)
    C = O.sample_BtNB(g, b_l, ninv, R, pairs)
    D = O.sample_D(g, d_l, None, pairs)
    M = BR.btnb_sparse(g, b_l, ninv, R)
    assert _gate(C, BR.extract_blocks(M, g, pairs), pairs) < 1e-12
    Dm = BR.local_operator_sparse(g, d_l)
    assert _gate(D, BR.extract_blocks(Dm, g, pairs), pairs) < 1e-12
    # the product vanishes beyond two tile hops
    rp, col = g.adjacency()
    two_hop = [set() for _ in range(g.ntiles)]
    for J in range(g.ntiles):
        for I in col[rp[J]:rp[J + 1]]:
            two_hop[J].update(col[rp[I]:rp[I + 1]].tolist())
    Mc = M.tocoo()
    k2 = k * k
    for i, j, v in zip(Mc.row, Mc.col, Mc.data):
        if v != 0.0:
            assert j // k2 in two_hop[i // k2]


@pytest.mark.parametrize("lmax,k,margin", TRANSITION_GRIDS)
def test_two_hop_blocks_match_dense_brute_force(lmax, k, margin):
    """The two-hop list covers every nonzero of the brute-force product, and
    the oracle's blocks on it (one-hop blocks included) equal the product's."""
    g = G.make_grid(lmax, k, polar_margin=margin)
    ninv, b_l, R = _inputs(g, seed=11)
    pairs = O.two_hop_block_list(g)
    assert set(O.stored_block_list(g)) <= set(pairs)
    M = BR.btnb_sparse(g, b_l, ninv, R)
    C = O.sample_BtNB(g, b_l, ninv, R, pairs)
    assert _gate(C, BR.extract_blocks(M, g, pairs), pairs) < 1e-12
    k2 = k * k
    listed = set(pairs)
    Mc = M.tocoo()
    for i, j, v in zip(Mc.row, Mc.col, Mc.data):
        J, K = i // k2, j // k2
        if v != 0.0 and K >= J:
            assert (J, K) in listed


def test_lmax64_btnb_matches_sparse_brute_force(lmax64_grid):
    g = lmax64_grid
    cfg = S.CONFIGS["lmax64"]
    ring, pin, nr, phi = g.pixel_coords()
    ninv = S.ninv_for(cfg, g.theta[ring], phi)
    b_l, R = S.gaussian_beam(cfg.lmax, g.npix, cfg.fwhm_pix)
    pairs = O.stored_block_list(g)
    C = O.sample_BtNB(g, b_l, ninv, R, pairs)
    M = BR.btnb_sparse(g, b_l, ninv, R)
    assert _gate(C, BR.extract_blocks(M, g, pairs), pairs) < 1e-12


def test_delta_map_gives_rank_one_blocks():
    """N^-1 = e_p: C_JK[a, b] = B(p, J_a) B(p, K_b) exactly (Eq. 15 closed form)."""
    g = G.make_grid(*TRANSITION_GRIDS[2][:2], polar_margin=TRANSITION_GRIDS[2][2])
    _, b_l, R = _inputs(g)
    Bs = BR.local_operator_sparse(g, b_l, R).tocsr()
    pairs = O.stored_block_list(g)
    k2 = g.k ** 2
    for p in (0, g.npix // 3, g.npix - 1):
        w = np.zeros(g.npix)
        w[p] = 1.0
        C = O.sample_BtNB(g, b_l, w, R, pairs)
        row = Bs[p].toarray().ravel()
        for n, (J, K) in enumerate(pairs):
            ref = np.outer(row[J * k2:(J + 1) * k2], row[K * k2:(K + 1) * k2])
            assert np.max(np.abs(C[n] - ref)) <= 1e-12 * max(1e-300, np.abs(row).max() ** 2)


def test_linearity_in_ninv():
    g = G.make_grid(32, 2, polar_margin=0.0)
    n1, b_l, R = _inputs(g, 1)
    n2, _, _ = _inputs(g, 2)
    pairs = O.stored_block_list(g)
    C1 = O.sample_BtNB(g, b_l, n1, R, pairs)
    C2 = O.sample_BtNB(g, b_l, n2, R, pairs)
    C12 = O.sample_BtNB(g, b_l, 0.3 * n1 - 1.7 * n2, R, pairs)
    assert np.max(np.abs(C12 - (0.3 * C1 - 1.7 * C2))) < 1e-14 * np.abs(C12).max() * 10


def test_blocks_are_symmetric_across_the_diagonal(lmax64_grid):
    """D_JK = D_KJ^T and C_JK = C_KJ^T, with the (K, J) blocks built from their
    own symmetry keys."""
    g = lmax64_grid
    rng = np.random.default_rng(3)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    b_l, R = S.gaussian_beam(g.lmax, g.npix, 3.0)
    opD = O.LocalOperator(g, S.prior(g.lmax))
    opB = O.LocalOperator(g, b_l, R)
    for J, K in O.stored_block_list(g)[::7]:
        assert np.array_equal(opD.block(J, K), opD.block(K, J).T) or \
            np.max(np.abs(opD.block(J, K) - opD.block(K, J).T)) < 1e-12 * np.abs(opD.block(J, J)).max()
        a = O.btnb_block(opB, ninv, J, K)
        b = O.btnb_block(opB, ninv, K, J)
        assert np.max(np.abs(a - b.T)) < 1e-13 * np.abs(a).max()


def test_rotation_equivariance():
    """Rotating the sky by 2 pi / g (g = gcd of all tile counts) moves every tile
    by T/g within its band; C(rotated N^-1) must be C(N^-1) with blocks moved."""
    g = G.make_grid(34, 2, polar_margin=2.0)          # tile counts 8, 24, 32, 40: gcd 8
    from math import gcd
    from functools import reduce
    gg = reduce(gcd, g.band_tiles)
    assert gg > 1
    k2 = g.k ** 2

    def rot_tile(t):
        b = g.tile_band(t)
        T = g.band_tiles[b]
        return g.band_tile0[b] + (t - g.band_tile0[b] + T // gg) % T

    perm = np.zeros(g.npix, dtype=np.int64)           # new pixel index of old pixel
    for t in range(g.ntiles):
        perm[t * k2:(t + 1) * k2] = rot_tile(t) * k2 + np.arange(k2)
    ninv, b_l, R = _inputs(g)
    rot = np.empty_like(ninv)
    rot[perm] = ninv
    opB = O.LocalOperator(g, b_l, R)
    opB2 = O.LocalOperator(g, b_l, R)
    for J, K in O.stored_block_list(g)[::5]:
        a = O.btnb_block(opB, ninv, J, K)
        b = O.btnb_block(opB2, rot, rot_tile(J), rot_tile(K))
        assert np.max(np.abs(a - b)) < 1e-13 * np.abs(a).max()


def test_north_south_mirror():
    """The grid is symmetric under theta -> pi - theta: D blocks of a northern
    band pair equal those of the mirrored southern pair with the ring index
    inside the tile reversed (r -> k-1-r, since rings run by increasing theta)."""
    g = G.make_grid(34, 2, polar_margin=2.0)
    k = g.k
    op = O.LocalOperator(g, S.prior(g.lmax))
    perm = np.array([c * k + (k - 1 - r) for c in range(k) for r in range(k)])
    n = g.nbands_hemi
    for i in range(n - 1):
        bN, bS = 2 * i, 2 * i + 1
        bN2, bS2 = 2 * (i + 1), 2 * (i + 1) + 1
        I_N, I_S = g.band_tile0[bN], g.band_tile0[bS]
        for dt in range(2):
            J_N, J_S = g.band_tile0[bN2] + dt, g.band_tile0[bS2] + dt
            a = op.block(I_N, J_N)
            b = op.block(I_S, J_S)[np.ix_(perm, perm)]
            assert np.max(np.abs(a - b)) < 1e-12 * np.abs(a).max()


def test_unique_key_reuse_matches_direct_evaluation():
    """Every cached block equals a fresh evaluation of its own tile pair."""
    g = G.make_grid(34, 2, polar_margin=2.0)
    b_l, R = S.gaussian_beam(g.lmax, g.npix, 3.0)
    op = O.LocalOperator(g, b_l, R)
    from oracle.kernel import legendre_series_in_y
    yR = O.radius_to_y(R)
    rp, col = g.adjacency()
    for I in range(0, g.ntiles, 3):
        for J in col[rp[I]:rp[I + 1]]:
            y = O.block_y(g, I, int(J))
            ref = np.where(y <= yR, legendre_series_in_y(b_l, y), 0.0)
            assert np.max(np.abs(op.block(I, int(J)) - ref)) <= 1e-13 * np.abs(ref).max()


# --- pixel-domain convolution (Section 4.1) ------------------------------------

@pytest.mark.parametrize("lmax,k,margin", TRANSITION_GRIDS)
def test_convolution_matches_sparse_brute_force(lmax, k, margin):
    """g = B-hat f blockwise (symmetry-keyed blocks, haversine geometry) equals
    the product with the operator assembled pair by pair from unit vectors."""
    g = G.make_grid(lmax, k, polar_margin=margin)
    rng = np.random.default_rng(lmax + k)
    f = rng.standard_normal(g.npix)
    b_l, R = S.gaussian_beam(lmax, g.npix, 2.0)
    got = O.convolve(g, b_l, f, R).ravel()
    want = BR.local_operator_sparse(g, b_l, R) @ f
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_lmax64_convolution_matches_sparse_brute_force(lmax64_grid):
    g = lmax64_grid
    rng = np.random.default_rng(5)
    f = rng.uniform(-1.0, 1.0, g.npix)
    b_l, R = S.gaussian_beam(g.lmax, g.npix, 3.0)
    got = O.convolve(g, b_l, f, R).ravel()
    want = BR.local_operator_sparse(g, b_l, R) @ f
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_convolution_is_self_adjoint_and_linear():
    """b(n_i . n_j) is symmetric in i, j, so <h, B f> = <B h, f>; and B is linear."""
    g = G.make_grid(34, 2, polar_margin=2.0)
    rng = np.random.default_rng(8)
    f, h = rng.standard_normal((2, g.npix))
    b_l, R = S.gaussian_beam(34, g.npix, 3.0)
    Bf = O.convolve(g, b_l, f, R).ravel()
    Bh = O.convolve(g, b_l, h, R).ravel()
    assert abs(h @ Bf - Bh @ f) <= 1e-12 * (np.abs(h) @ np.abs(Bf))
    B2 = O.convolve(g, b_l, 2.0 * f - 3.0 * h, R).ravel()
    assert np.abs(B2 - (2.0 * Bf - 3.0 * Bh)).max() <= 1e-12 * np.abs(B2).max()
