"""Pins for the oracle's two-grid operator B-hat = Y_2 B Y_1^T (Eqs. 13 and
16) and B-hat^T N_2^-1 B-hat (Eq. 15): the tile relation against an
independent floating-point location of tile centres, every block and the product against
a dense per-pair brute force on small grid pairs (including tile sizes that
differ, so the blocks are rectangular), the band limit of the kernel against
the addition theorem, and the limit Y_2 = Y_1, which must reproduce the
one-grid operator bit for bit."""
import numpy as np
import pytest
import scipy.special as ss

from oracle import brute as BR
from oracle import grid as G
from oracle import operators as O
from oracle import twogrid as X
from workloads import synth as S

# (grid 2, grid 1) as (lmax, k, margin): finer auxiliary grids, tile-count
# transitions on both sides, and tile sizes that differ
PAIRS = [((34, 2, None), (16, 2, None)),
         ((32, 2, 0.0), (20, 2, 0.0)),
         ((40, 4, None), (20, 2, None)),
         ((16, 2, None), (34, 2, 2.0))]


def _grids(pair):
    (l2, k2, m2), (l1, k1, m1) = pair
    return G.make_grid(l2, k2, polar_margin=m2), G.make_grid(l1, k1, polar_margin=m1)


def _gate(C, ref, pairs):
    rowmax = {}
    for n, (J, K) in enumerate(pairs):
        rowmax[J] = max(rowmax.get(J, 0.0), np.abs(ref[n]).max())
    return max(np.abs(C[n] - ref[n]).max() / rowmax[J] for n, (J, K) in enumerate(pairs))


@pytest.mark.parametrize("pair", PAIRS)
def test_relation_matches_floating_point_centre_location(pair):
    g2, g1 = _grids(pair)
    rp, col = X.cross_adjacency(g2, g1)
    got = np.zeros((g2.ntiles, g1.ntiles), dtype=bool)
    for I in range(g2.ntiles):
        got[I, col[rp[I]:rp[I + 1]]] = True
    assert np.array_equal(got, BR.cross_relation_dense(g2, g1))
    assert got.any(axis=0).all() and got.any(axis=1).all()     # every tile has a partner
    assert [X.tile_centre_container(g2, g1, I) for I in range(g2.ntiles)] == X.centre_containers(g2, g1).tolist()


def test_band_ranges_contain_their_rings():
    """Each ring's colatitude lies strictly inside its band's range (the
    Gauss-Legendre zeros interlace with j pi / R)."""
    for lmax, k in [(16, 2), (64, 8), (255, 8), (3000, 8)]:
        g = G.make_grid(lmax, k)
        for b, rings in enumerate(g.band_rings):
            lo, hi, den = X.band_colatitude(g, b)
            th = g.theta[rings] / np.pi
            assert np.all(th > lo / den) and np.all(th < hi / den)


@pytest.mark.parametrize("lmax,k,margin", [(20, 2, 0.0), (34, 2, 2.0), (64, 8, None), (100, 8, None)])
def test_equal_grids_reproduce_the_one_grid_operator(lmax, k, margin):
    """Y_2 = Y_1: the relation is the one-grid adjacency and every block and
    every product block is bitwise the one-grid oracle's."""
    g = G.make_grid(lmax, k, polar_margin=margin)
    for J in range(g.ntiles):
        assert X.cross_neighbours(g, g, J) == g.tile_neighbours(J)
    rng = np.random.default_rng(4)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    pairs = O.stored_block_list(g)
    if len(pairs) > 400:
        pairs = [pairs[i] for i in sorted(rng.choice(len(pairs), 400, replace=False))]
    C1 = O.sample_BtNB(g, b_l, ninv, R, pairs)
    C2 = X.sample_BtNB_cross(g, g, b_l, ninv, R, pairs)
    assert np.array_equal(C1, C2)
    op1, op2 = O.LocalOperator(g, b_l, R), X.CrossOperator(g, g, b_l, R)
    for J, K in pairs[:100]:
        assert np.array_equal(op1.block(J, K), op2.block(J, K))


@pytest.mark.parametrize("pair", PAIRS)
def test_blocks_and_product_match_dense_brute_force(pair):
    g2, g1 = _grids(pair)
    rng = np.random.default_rng(9)
    ninv2 = rng.uniform(0.5, 2.0, g2.npix)
    ninv2[rng.random(g2.npix) < 0.1] = 0.0
    b_l, R = S.gaussian_beam(g1.lmax, g1.npix, 3.0)
    Bd = BR.cross_operator_dense(g2, g1, b_l, R)           # Npix_2 x Npix_1
    k22, k12 = g2.k ** 2, g1.k ** 2
    # every block of the relation, in cross-adjacency order
    blocks = X.sample_B_cross(g2, g1, b_l, R)
    rp, col = X.cross_adjacency(g2, g1)
    assert blocks.shape[1:] == (k22, k12)
    peak = np.abs(Bd).max()
    n = 0
    for I in range(g2.ntiles):
        for J in col[rp[I]:rp[I + 1]]:
            ref = Bd[I * k22:(I + 1) * k22, int(J) * k12:(int(J) + 1) * k12]
            assert np.abs(blocks[n] - ref).max() <= 1e-13 * peak
            n += 1
    assert n == blocks.shape[0]
    # the product on the stored pattern of Y_1, and zero where no tile of Y_2 meets both
    Cd = Bd.T @ (ninv2[:, None] * Bd)
    pairs = O.stored_block_list(g1)
    C = X.sample_BtNB_cross(g2, g1, b_l, ninv2, R, pairs)
    ref = np.stack([Cd[J * k12:(J + 1) * k12, K * k12:(K + 1) * k12] for J, K in pairs])
    assert _gate(C, ref, pairs) < 1e-12
    op = X.CrossOperator(g2, g1, b_l, R)
    # stored blocks with an empty sum (Y_2 the coarser grid) are exact zeros
    empty = [n for n, (J, K) in enumerate(pairs) if not set(op.neighbours(J)) & set(op.neighbours(K))]
    assert all(not C[n].any() for n in empty)
    if g2.lmax < g1.lmax:
        assert empty, "a coarser auxiliary grid leaves some stored blocks without terms"
    for J in range(g1.ntiles):
        for K in range(g1.ntiles):
            if not set(op.neighbours(J)) & set(op.neighbours(K)):
                assert not Cd[J * k12:(J + 1) * k12, K * k12:(K + 1) * k12].any()


def test_kernel_band_limit_is_the_smaller_lmax():
    """B-hat = Y_2 B Y_1^T passes only l <= min(lmax_1, lmax_2): with b_l = 1
    up to the larger band limit, an element equals the addition-theorem sum
    over l <= the smaller one (and not over l <= the larger)."""
    g1 = G.make_grid(3, 2)
    g2 = G.make_grid(9, 2)
    op = X.CrossOperator(g2, g1, np.ones(10), None)
    ring2, _, _, phi2 = g2.pixel_coords()
    ring1, _, _, phi1 = g1.pixel_coords()
    k22, k12 = g2.k ** 2, g1.k ** 2
    checked = 0
    for J in range(0, g1.ntiles, 3):
        for I in op.neighbours(J)[:2]:
            blk = op.block(I, J)
            for a, b in [(0, 0), (k22 - 1, k12 - 1), (1, 2)]:
                p, q = I * k22 + a, J * k12 + b
                th2, ph2 = g2.theta[ring2[p]], phi2[p]
                th1, ph1 = g1.theta[ring1[q]], phi1[q]

                def harm(L):
                    return sum((ss.sph_harm_y(l, m, th2, ph2) * np.conj(ss.sph_harm_y(l, m, th1, ph1))).real
                               for l in range(L + 1) for m in range(-l, l + 1))
                assert abs(blk[a, b] - harm(3)) < 1e-13 * 16
                assert abs(blk[a, b] - harm(9)) > 1e-3
                checked += 1
    assert checked >= 6


def test_delta_map_gives_rank_one_blocks_and_linearity():
    g2, g1 = _grids(PAIRS[0])
    b_l, R = S.gaussian_beam(g1.lmax, g1.npix, 3.0)
    op = X.CrossOperator(g2, g1, b_l, R)
    k22 = g2.k ** 2
    p = 37 * k22 + 2
    w = np.zeros(g2.npix)
    w[p] = 1.0
    pairs = O.stored_block_list(g1)
    C = X.sample_BtNB_cross(g2, g1, b_l, w, R, pairs)
    I, a = divmod(p, k22)
    peak = max(np.abs(op.block(I, J)).max() for J in range(g1.ntiles)) ** 2
    nonzero = 0
    for n, (J, K) in enumerate(pairs):
        ref = np.outer(op.block(I, J)[a], op.block(I, K)[a])     # zero unless I meets both
        assert np.abs(C[n] - ref).max() <= 1e-14 * peak
        nonzero += bool(ref.any())
    assert nonzero > 0
    rng = np.random.default_rng(1)
    w1, w2 = rng.uniform(0.5, 2, g2.npix), rng.uniform(0.5, 2, g2.npix)
    C1 = X.sample_BtNB_cross(g2, g1, b_l, w1, R, pairs)
    C2 = X.sample_BtNB_cross(g2, g1, b_l, w2, R, pairs)
    C12 = X.sample_BtNB_cross(g2, g1, b_l, 0.3 * w1 - 1.7 * w2, R, pairs)
    assert np.abs(C12 - (0.3 * C1 - 1.7 * C2)).max() < 1e-13 * np.abs(C12).max()
