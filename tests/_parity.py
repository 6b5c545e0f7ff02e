"""Helpers shared by the GPU parity tests: error metrics and sampled oracle
comparisons.  The oracle is imported here only to compute expected values."""
from __future__ import annotations

import numpy as np

from oracle import grid as G
from oracle import operators as O
from workloads import synth as S


def gate(C, ref, rows):
    """max |C - ref| / M_J with M_J the largest |ref| over the compared blocks of
    block-row J (rows[n] is the J of block n); infinite if any value is not
    finite (a NaN would otherwise drop out of the maximum)."""
    if not (np.isfinite(C).all() and np.isfinite(ref).all()):
        return float("inf")
    rows = np.asarray(rows)
    mj = {}
    for n, J in enumerate(rows):
        mj[J] = max(mj.get(J, 0.0), float(np.abs(ref[n]).max()))
    worst = 0.0
    for n, J in enumerate(rows):
        if mj[J] > 0:
            worst = max(worst, float(np.abs(C[n] - ref[n]).max()) / mj[J])
        else:
            worst = max(worst, float(np.abs(C[n]).max()))
    return worst


def error_report(C, ref, rows):
    """Per-element |C - ref| / max(|ref|, 1e-8 M_J): median, p99, max."""
    rows = np.asarray(rows)
    mj = {}
    for n, J in enumerate(rows):
        mj[J] = max(mj.get(J, 0.0), float(np.abs(ref[n]).max()))
    scale = np.array([mj[J] for J in rows])[:, None, None]
    # rows whose blocks are all zero (fully masked N^-1) compare absolutely
    with np.errstate(invalid="ignore"):
        rel = np.abs(C - ref) / np.maximum(np.maximum(np.abs(ref), 1e-8 * scale), 1e-300)
    return {"median": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
            "max": float(rel.max()), "gate": gate(C, ref, rows),
            "nonfinite": int(np.size(C) - np.count_nonzero(np.isfinite(C)))}


def stored_pairs(g: G.Grid):
    return O.stored_block_list(g)


def sample_rows(g: G.Grid, n_random: int, seed: int):
    """Block-rows J to compare at full size: two tiles (the first and a random
    one) of the polar bands, the equatorial bands, up to four bands whose tile
    count differs from a neighbour's and four random bands, plus n_random
    random tiles anywhere."""
    rng = np.random.default_rng(seed)
    nb = len(g.band_tiles)
    bands = {0, 1, nb - 2, nb - 1}
    trans = [b for b in range(nb) if any(g.band_tiles[x] != g.band_tiles[b] for x in g.band_neighbours(b))]
    bands.update(trans[:4])
    bands.update(rng.choice(nb, size=min(nb, 4), replace=False).tolist())
    rows = set()
    for b in bands:
        t0 = g.band_tile0[b]
        rows.update([t0, t0 + int(rng.integers(g.band_tiles[b]))])
    rows.update(rng.choice(g.ntiles, size=n_random, replace=False).tolist())
    return sorted(int(r) for r in rows)


def block_index(og: G.Grid, blk_ptr, blk_col, rows):
    """Stored-block indices and (J, K) pairs of the given block-rows, taken from
    the library's block CSR after checking each row against the oracle's own
    neighbour list (so the layout is verified at full size too)."""
    idx, pairs = [], []
    for J in rows:
        ks = [K for K in og.tile_neighbours(J) if K >= J]
        got = blk_col[blk_ptr[J]:blk_ptr[J + 1]].tolist()
        assert got == ks, f"stored-block row {J}: library {got} oracle {ks}"
        for n, K in zip(range(blk_ptr[J], blk_ptr[J + 1]), ks):
            idx.append(int(n))
            pairs.append((J, K))
    return np.asarray(idx), pairs


def config_inputs(cfg: S.Config, g_oracle: G.Grid):
    ring, pin, nr, phi = g_oracle.pixel_coords()
    ninv = S.ninv_for(cfg, g_oracle.theta[ring], phi)
    b_l, R = S.gaussian_beam(cfg.lmax, g_oracle.npix, cfg.fwhm_pix)
    return ninv, b_l, R, S.prior(cfg.lmax)
