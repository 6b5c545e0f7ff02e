"""Writes tests/golden/table1_npix.txt: the grid sizes every reading of the
ambiguous parts of Fig. 3 / Section 2.5 gives, next to every grid size the
paper prints.  Calls only the oracle (oracle.grid); run from the repository
root:  python tests/golden/make_grid_readings.py

Readings enumerated (the fields of oracle.grid.Readings):
  alpha_ring   ring of north band i that fixes alpha_i: "pole" (ring i k, as
               Fig. 3 writes theta_{ik}) or "equator" (ring i k + k - 1, the
               "southmost ring" of Section 2.5).  Taking the largest alpha
               over the band's k rings is the same as "equator": the ring
               lengths Eq. 3 asks for grow towards the equator.
  alpha_m      the m of alpha = ceil((2m + 1) / k): the smallest m satisfying
               Eq. 3 (Fig. 3) or one less (the largest m kept, Section 2.1).
  t0_rule      T_0 the smallest 5-smooth number ">=" alpha_0 (Fig. 3) or ">"
               (Section 2.5).
  upper_rule   t <= 3 alpha (Fig. 3) or t < 3 alpha (Section 2.5).
  band1        band 1 may change its tile count ("allow", the caption of
               Fig. 3) or not ("forbid", the -1 sentinel taken literally).
Margin: the right-hand side of Eq. 3, max(100, lmax/100) in the paper; the
scan covers every integer margin in [-30, 120].

Printed sizes: Table 1 (SymPix, k = 8): lmax 511 -> 390,656; 639 -> 591,232;
767 -> 838,656.  Section 3.1: lmax 2000, k = 4 -> 5.6e6 (two significant
figures).  Section 3.2: lmax 735, k = 8 -> about 780,000.
"""
from __future__ import annotations

import itertools
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import grid as G  # noqa: E402

OUT = os.path.join(HERE, "table1_npix.txt")

TABLE1 = ((511, 8, 390656), (639, 8, 591232), (767, 8, 838656))
SEC31 = (2000, 4, 5.6e6)        # two significant figures
SEC32 = (735, 8, 780000)        # "about"
MARGINS = range(-30, 121)


def all_readings():
    for ring, m, t0, up, b1 in itertools.product(("pole", "equator"), ("first_omitted", "max_kept"),
                                                 (">=", ">"), ("<=", "<"), (True, False)):
        yield G.Readings(alpha_ring=ring, alpha_m=m, t0_rule=t0, upper_rule=up, allow_first_change=b1)


def reading_name(rd: G.Readings) -> str:
    return (f"{rd.alpha_ring}/{rd.alpha_m}/T0{rd.t0_rule}/t{rd.upper_rule}3a/"
            f"band1-{'allow' if rd.allow_first_change else 'forbid'}")


_rings = {}


def _ring_table(lmax, k):
    if (lmax, k) not in _rings:
        nrings = -(-(lmax + 1) // (2 * k)) * 2 * k
        _, s, c, _ = G.gauss_legendre_theta(nrings)
        _rings[(lmax, k)] = (nrings // (2 * k), s, c)
    return _rings[(lmax, k)]


def grid_size(lmax, k, rd, margin=None):
    """(npix of the tile programme or None if infeasible, 2 k^2 sum alpha_i)
    for one reading and margin; the oracle's own steps (Eq. 3, Fig. 3)."""
    n, s, c = _ring_table(lmax, k)
    thr = G.polar_threshold(lmax) if margin is None else float(margin)
    alpha = G.alpha_per_band(lmax, k, s, c, n, thr, rd)
    tiles = G.optimal_tiles(alpha, rd)
    npix = None if tiles is None else 2 * k * k * sum(tiles)
    return npix, 2 * k * k * sum(alpha)


def paper_margin_rows():
    """One row per reading at the paper's margin: npix at the five printed
    cases, and 2 k^2 sum(alpha) (a lower bound of npix, since T_i >= alpha_i)
    at the Table 1 cases."""
    rows = []
    for rd in all_readings():
        sizes, lower = [], []
        for lmax, k, _ in TABLE1 + (SEC31, SEC32):
            npix, low = grid_size(lmax, k, rd)
            sizes.append(npix)
            lower.append(low)
        rows.append((reading_name(rd), sizes, lower[:3]))
    return rows


def margin_scan_row(rd):
    """For one reading: per Table 1 case the margins in [-30, 120] whose grid
    has the printed size, and the nearest size with its margin."""
    out = []
    for lmax, k, printed in TABLE1:
        hits, best = [], None
        for mg in MARGINS:
            npix, _ = grid_size(lmax, k, rd, mg)
            if npix is None:
                continue
            if npix == printed:
                hits.append(mg)
            d = abs(npix - printed)
            if best is None or d < best[0]:
                best = (d, npix, mg)
        out.append((hits, best))
    return out


def fmt(v):
    return "infeasible" if v is None else str(v)


def write(path=OUT):
    lines = ["# Written by tests/golden/make_grid_readings.py, which calls only oracle/ (do not edit by hand).",
             "# Grid sizes of every reading of Fig. 3 / Section 2.5 next to every size the paper prints.",
             "# printed: Table 1 (k=8) 511 -> 390656, 639 -> 591232, 767 -> 838656;",
             "#          Section 3.1 (2000, k=4) -> 5.6e6 (2 s.f.); Section 3.2 (735, k=8) -> about 780000.",
             "[paper_margin]",
             "# reading | npix 511 639 767 (2000,4) (735,8) | 2k^2*sum(alpha) 511 639 767"]
    for name, sizes, lower in paper_margin_rows():
        lines.append(f"{name} | {' '.join(fmt(v) for v in sizes)} | {' '.join(str(v) for v in lower)}")
    lines += ["[margin_scan]",
              "# reading | per Table 1 case: margins in [-30,120] with the printed size (or -), "
              "then nearest size@margin"]
    common = []
    for rd in all_readings():
        cells, sets = [], []
        for hits, best in margin_scan_row(rd):
            sets.append(set(hits))
            h = ",".join(str(m) for m in hits) if hits else "-"
            cells.append(f"{h} {best[1]}@{best[2]}" if best else f"{h} infeasible")
        both = sorted(set.intersection(*sets))
        if both:
            common.append((reading_name(rd), both))
        lines.append(f"{reading_name(rd)} | " + " | ".join(cells))
    lines += ["[summary]",
              "readings_matching_all_table1_at_one_margin " + (
                  "; ".join(f"{n}@{m}" for n, m in common) if common else "none")]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return lines


def parse(path=OUT):
    """The golden file as {"paper_margin": {name: (sizes, lower)}, "margin_scan":
    {name: [(hits, nearest, margin)]}, "summary": str}."""
    sec, out = None, {"paper_margin": {}, "margin_scan": {}, "summary": ""}
    for line in open(path):
        line = line.rstrip("\n")
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            sec = line.strip("[]")
            continue
        if sec == "paper_margin":
            name, a, b = [x.strip() for x in line.split("|")]
            sizes = [None if v == "infeasible" else int(v) for v in a.split()]
            out["paper_margin"][name] = (sizes, [int(v) for v in b.split()])
        elif sec == "margin_scan":
            parts = [x.strip() for x in line.split("|")]
            cells = []
            for cell in parts[1:]:
                h, nb = cell.split()
                hits = [] if h == "-" else [int(v) for v in h.split(",")]
                if nb == "infeasible":
                    cells.append((hits, None, None))
                else:
                    v, m = nb.split("@")
                    cells.append((hits, int(v), int(m)))
            out["margin_scan"][parts[0]] = cells
        elif sec == "summary":
            out["summary"] = line
    return out


if __name__ == "__main__":
    for line in write():
        print(line)
