"""Oracle: the SymPix grid (test infrastructure only; see package docstring).

Follows Section 2 of the paper: Gauss-Legendre ring latitudes (Section 2.1),
the polar-optimisation cut of Eq. 3, the dynamic-programming choice of tiles
per band (Fig. 3, Eqs. 4-5, Section 2.5), the memory layout of Section 2.4 and
the neighbouring-tile relation of Section 2.2.

Where the paper is ambiguous the reading used is a field of ``Readings``; the
defaults are the readings the build uses.  No combination of the readings, at
any margin of Eq. 3 in [-30, 120], reproduces the SymPix pixel counts printed
in Table 1: tests/golden/make_grid_readings.py (which calls only this module)
records every reading's sizes next to the printed ones in
tests/golden/table1_npix.txt.  With the paper's margin, 2 k^2 sum(alpha_i)
alone exceeds each printed count, so no tile programme over these alpha can
reach them.  The defaults follow Fig. 3 literally, except that band 1 may
differ from band 0 as the caption of Fig. 3 allows (taken literally, the
sentinel makes every printed case infeasible).  The tile-count optimisation is
therefore "parity unpinned" against Table 1; it is pinned instead by a closed
form (every band at the same count when Eq. 3 never holds), by brute force
with the run rule switched off, and by the structural rules of Section 2.3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# Gauss-Legendre rings (Section 1 and 2.1; Fig. 3 "as for Gauss-Legendre grid")
# ---------------------------------------------------------------------------

def legendre_pair_in_y(n: int, y: np.ndarray):
    """Return (P_n(1-y), P_{n-1}(1-y)) for n >= 1.

    Uses the three-term Legendre recurrence rewritten in y = 1 - x, carrying
    D_l = P_l - P_{l-1}:  D_1 = -y,  (l+1) D_{l+1} = l D_l - (2l+1) y P_l,
    P_{l+1} = P_l + D_{l+1}.  This avoids forming x = cos(theta) near the
    poles, where 1 - x would lose all relative precision.
    """
    y = np.asarray(y, dtype=np.float64)
    p_prev = np.ones_like(y)          # P_0
    d = -y                            # D_1
    p = p_prev + d                    # P_1
    for l in range(1, n):
        d = (l * d - (2 * l + 1) * y * p) / (l + 1)
        p_prev = p
        p = p + d
    return p, p_prev


def gauss_legendre_theta(nrings: int):
    """Colatitudes theta_j (j = 0 at the north pole) with P_nrings(cos theta_j) = 0,
    and the Gauss-Legendre weights w_j (Eq. 2).

    Newton iteration in theta on f(theta) = P_N(cos theta), whose derivative is
    f'(theta) = -N (P_{N-1} - x P_N) / sin(theta).  Only the northern half is
    solved; the south is the mirror image theta -> pi - theta (nrings is even).
    Returns (theta, sin_theta, cos_theta, weight), each of length nrings.
    """
    n = int(nrings)
    if n < 2 or n % 2:
        raise ValueError("nrings must be even and >= 2")
    half = n // 2
    j = np.arange(half, dtype=np.float64)
    theta = np.pi * (4.0 * j + 3.0) / (4.0 * n + 2.0)   # classical start value

    def newton_step(th):
        y = 2.0 * np.sin(0.5 * th) ** 2
        x = np.cos(th)
        pn, pn1 = legendre_pair_in_y(n, y)
        return pn * np.sin(th) / (n * (pn1 - x * pn))

    # Rounding in P_N makes the last step flip by about one ulp, so stop once
    # every step is within a few ulps and then take one polish step.
    for _ in range(100):
        step = newton_step(theta)
        theta = theta + step
        if np.all(np.abs(step) <= 4.0 * np.finfo(np.float64).eps * theta):
            break
    else:  # pragma: no cover - convergence is quadratic from these start values
        raise RuntimeError("Gauss-Legendre Newton iteration did not converge")
    theta = theta + newton_step(theta)     # one polish step

    y = 2.0 * np.sin(0.5 * theta) ** 2
    _, pn1 = legendre_pair_in_y(n, y)
    s = np.sin(theta)
    c = np.cos(theta)
    w = 2.0 * s * s / (n * pn1) ** 2

    full_theta = np.concatenate([theta, (np.pi - theta)[::-1]])
    full_sin = np.concatenate([s, s[::-1]])
    full_cos = np.concatenate([c, -c[::-1]])
    full_w = np.concatenate([w, w[::-1]])
    return full_theta, full_sin, full_cos, full_w


# ---------------------------------------------------------------------------
# Readings of the ambiguous parts of Fig. 3 / Section 2.5
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Readings:
    # Which ring of north band i fixes alpha_i: "pole" = ring i*k (Fig. 3),
    # "equator" = ring i*k+k-1 (the "southmost ring" of the prose).
    alpha_ring: str = "pole"
    # "first_omitted": m is the smallest m satisfying Eq. 3 (Fig. 3 literally);
    # "max_kept": m is one less (the largest m kept, prose of Section 2.1).
    alpha_m: str = "first_omitted"
    # T_0 is the smallest 5-smooth number ">=" alpha_0 (Fig. 3) or ">" (prose).
    t0_rule: str = ">="
    # Upper bound t <= 3 alpha (Fig. 3) or t < 3 alpha (prose).
    upper_rule: str = "<="
    # Whether band 1 may differ from band 0 (Fig. 3 caption) or not (the -1
    # sentinel taken literally).
    allow_first_change: bool = True


DEFAULT_READINGS = Readings()

RATIOS = ((3, 1), (2, 1), (1, 1), (4, 3), (5, 4), (6, 5))   # listed order of Fig. 3


def polar_threshold(lmax: int) -> float:
    """The right-hand side of Eq. 3: max(100, 0.01 lmax)."""
    return max(100.0, 0.01 * lmax)


def min_m_eq3(lmax: int, sin_t: float, cos_t: float, thr: float):
    """Smallest integer m in [0, lmax] satisfying Eq. 3 at a ring with the given
    sin/cos of its colatitude, or None if none does.  A negative radicand
    m^2 - 2 m cos(theta) counts as not satisfying the inequality."""
    for m in range(0, lmax + 1):
        rad = m * m - 2.0 * m * cos_t
        if rad < 0.0:
            continue
        if math.sqrt(rad) - lmax * sin_t > thr:
            return m
    return None


def alpha_per_band(lmax: int, k: int, sin_t, cos_t, nbands: int, thr: float,
                   rd: Readings = DEFAULT_READINGS):
    """alpha_i = ceil((2m + 1)/k) for each northern band i (Fig. 3)."""
    out = []
    for i in range(nbands):
        j = i * k if rd.alpha_ring == "pole" else i * k + k - 1
        m = min_m_eq3(lmax, float(sin_t[j]), float(cos_t[j]), thr)
        if m is None:
            m = lmax
        elif rd.alpha_m == "max_kept":
            m = m - 1
        out.append(-((-(2 * m + 1)) // k))   # integer ceil
    return out


def is_5_smooth(t: int) -> bool:
    for p in (2, 3, 5):
        while t % p == 0:
            t //= p
    return t == 1


def smallest_5_smooth(alpha: int, strict: bool) -> int:
    t = alpha + 1 if strict else max(alpha, 1)
    while not is_5_smooth(t):
        t += 1
    return t


def optimal_tiles(alpha, rd: Readings = DEFAULT_READINGS, enforce_runs: bool = True):
    """The dynamic programme of Fig. 3 over the cost of Eq. 4.

    C[i][t] is the best partial cost for bands 0..i with T_i = t, P[i][t] the
    T_{i-1} of that partial solution.  Band 0 is the smallest 5-smooth number
    not below alpha_0.  A band may change its tile count by a ratio of Eq. 5
    only if the previous band did not change (P[i-1][t_prev] == t_prev), which
    keeps runs of at least two equal bands; band 1 may change freely when
    ``allow_first_change``.  Ties keep the first candidate met with t_prev in
    ascending order and ratios in the listed order; the final argmin takes the
    smallest t.  Returns the list T_i, or None if no layout is feasible.

    ``enforce_runs=False`` drops the run rule; the programme is then an exact
    dynamic programme over (band, tile count) and tests compare it with brute
    force.  With the rule on, the single pointer per state makes the paper's
    programme a heuristic (it can miss a cheaper layout that obeys the rule).
    """
    n = len(alpha)
    t0 = smallest_5_smooth(alpha[0], strict=(rd.t0_rule == ">"))
    C = [dict() for _ in range(n)]
    P = [dict() for _ in range(n)]
    C[0][t0] = (t0 - alpha[0]) ** 2
    P[0][t0] = -1
    for i in range(1, n):
        a = alpha[i]
        hi = 3 * a
        for t_prev in sorted(C[i - 1]):
            c_prev = C[i - 1][t_prev]
            prev_ptr = P[i - 1][t_prev]
            for num, den in RATIOS:
                if (num * t_prev) % den:
                    continue
                t = num * t_prev // den
                if t < a:
                    continue
                if rd.upper_rule == "<=" and t > hi:
                    continue
                if rd.upper_rule == "<" and t >= hi:
                    continue
                steady = (prev_ptr == t_prev) or (num == den)
                if (i == 1 and rd.allow_first_change) or not enforce_runs:
                    steady = True
                if not steady:
                    continue
                cand = c_prev + (a - t) ** 2
                if cand < C[i].get(t, math.inf):
                    C[i][t] = cand
                    P[i][t] = t_prev
    if not C[n - 1]:
        return None
    best = min(C[n - 1].values())
    t_last = min(t for t, c in C[n - 1].items() if c == best)
    tiles = [0] * n
    tiles[n - 1] = t_last
    for i in range(n - 1, 0, -1):
        tiles[i - 1] = P[i][tiles[i]]
    return tiles


# ---------------------------------------------------------------------------
# The grid object: rings, bands in storage order, tiles and adjacency
# ---------------------------------------------------------------------------

@dataclass
class Grid:
    lmax: int
    k: int
    nrings: int
    nbands_hemi: int
    theta: np.ndarray          # [nrings], ring j from the north pole
    sin_theta: np.ndarray
    cos_theta: np.ndarray
    weight: np.ndarray
    alpha: list                # [n] per northern band
    tiles_north: list          # [n] T_i per northern band
    # storage order of bands: N0, S0, N1, S1, ...
    band_tiles: list = field(default_factory=list)     # [2n]
    band_alpha: list = field(default_factory=list)
    band_rings: list = field(default_factory=list)     # [2n] list of k ring indices, theta increasing
    band_pix0: list = field(default_factory=list)      # first pixel of each band
    band_tile0: list = field(default_factory=list)     # first global tile of each band
    npix: int = 0
    ntiles: int = 0

    # --- pixel geometry -------------------------------------------------
    def ring_npix(self):
        out = np.zeros(self.nrings, dtype=np.int64)
        for b, rings in enumerate(self.band_rings):
            for j in rings:
                out[j] = self.k * self.band_tiles[b]
        return out

    def ring_first_pix(self):
        """First pixel index of every ring (Section 2.4 layout: a ring's pixels
        are strided by k inside its band)."""
        out = np.zeros(self.nrings, dtype=np.int64)
        for b, rings in enumerate(self.band_rings):
            for r, j in enumerate(rings):
                out[j] = self.band_pix0[b] + r
        return out

    def tile_band(self, tile: int) -> int:
        return int(np.searchsorted(np.asarray(self.band_tile0), tile, side="right")) - 1

    def pixel_index(self, band: int, t: int, c: int, r: int) -> int:
        """Section 2.4: bands interleaved N0,S0,N1,...; inside a band tiles by
        increasing phi; inside a tile theta runs fastest (r), then column c."""
        k = self.k
        return self.band_pix0[band] + t * k * k + c * k + r

    def pixel_coords(self):
        """(ring index, ring-local pixel index p, n_ring, phi) for every pixel,
        with phi = 2 pi (p + 1/2) / n_ring (first pixel half a step from phi = 0)."""
        k = self.k
        ring = np.zeros(self.npix, dtype=np.int64)
        pin = np.zeros(self.npix, dtype=np.int64)
        nr = np.zeros(self.npix, dtype=np.int64)
        for b in range(len(self.band_tiles)):
            T = self.band_tiles[b]
            t, c, r = np.meshgrid(np.arange(T), np.arange(k), np.arange(k), indexing="ij")
            idx = self.band_pix0[b] + t * k * k + c * k + r
            ring[idx] = np.asarray(self.band_rings[b])[r]
            pin[idx] = t * k + c
            nr[idx] = k * T
        phi = 2.0 * np.pi * (pin + 0.5) / nr
        return ring, pin, nr, phi

    # --- tiles ------------------------------------------------------------
    def band_neighbours(self, b: int):
        """Latitudinally neighbouring bands of storage band b (no pole crossing;
        the two equatorial bands N_{n-1}, S_{n-1} neighbour each other)."""
        n = self.nbands_hemi
        i, south = divmod(b, 2)
        out = []
        if i > 0:
            out.append(2 * (i - 1) + south)
        if i < n - 1:
            out.append(2 * (i + 1) + south)
        else:
            out.append(2 * i + (1 - south))
        return out

    def tile_neighbours(self, tile: int):
        """Sorted global tile ids neighbouring ``tile`` (itself included).

        Same band: t-1, t, t+1 modulo T.  Neighbouring band: every tile whose
        closed phi interval [t'/T', (t'+1)/T'] meets [t/T, (t+1)/T] modulo 1,
        tested in exact integers after scaling by T*T'.
        """
        b = self.tile_band(tile)
        T = self.band_tiles[b]
        t = tile - self.band_tile0[b]
        out = {self.band_tile0[b] + ((t + d) % T) for d in (-1, 0, 1)}
        for b2 in self.band_neighbours(b):
            T2 = self.band_tiles[b2]
            lo1, hi1 = t * T2, (t + 1) * T2          # interval of tile t scaled by T*T2
            M = T * T2
            if T2 <= 8:
                cands = range(T2)
            else:
                cands = [u % T2 for u in range(t * T2 // T - 1, (t + 1) * T2 // T + 2)]
            for t2 in cands:
                lo2, hi2 = t2 * T, (t2 + 1) * T
                hit = False
                for shift in (-M, 0, M):
                    if lo1 <= hi2 + shift and lo2 + shift <= hi1:
                        hit = True
                        break
                if hit:
                    out.add(self.band_tile0[b2] + t2)
        return sorted(out)

    def adjacency(self):
        """Full tile adjacency as CSR (row_ptr int64, col int32)."""
        rows = [self.tile_neighbours(t) for t in range(self.ntiles)]
        row_ptr = np.zeros(self.ntiles + 1, dtype=np.int64)
        row_ptr[1:] = np.cumsum([len(r) for r in rows])
        col = np.fromiter((c for r in rows for c in r), dtype=np.int32, count=int(row_ptr[-1]))
        return row_ptr, col

    def stored_blocks(self):
        """The stored output blocks: pairs (J, K) with K a neighbour of J and
        K >= J, as CSR over J (row_ptr int64, col int32)."""
        rp, col = self.adjacency()
        rows = []
        for j in range(self.ntiles):
            rows.append([int(c) for c in col[rp[j]:rp[j + 1]] if c >= j])
        row_ptr = np.zeros(self.ntiles + 1, dtype=np.int64)
        row_ptr[1:] = np.cumsum([len(r) for r in rows])
        cols = np.fromiter((c for r in rows for c in r), dtype=np.int32, count=int(row_ptr[-1]))
        return row_ptr, cols


class InfeasibleGrid(ValueError):
    pass


def make_grid(lmax: int, k: int, polar_margin: float | None = None,
              rd: Readings = DEFAULT_READINGS) -> Grid:
    """Optimal-SymPix-Grid of Fig. 3 followed by the Section 2.4 layout."""
    if lmax < 1 or k < 1:
        raise ValueError("lmax and k must be >= 1")
    nrings = -(-(lmax + 1) // (2 * k)) * 2 * k      # lmax+1 rounded up to a multiple of 2k
    n = nrings // (2 * k)
    theta, s, c, w = gauss_legendre_theta(nrings)
    thr = polar_threshold(lmax) if polar_margin is None else float(polar_margin)
    alpha = alpha_per_band(lmax, k, s, c, n, thr, rd)
    tiles = optimal_tiles(alpha, rd)
    if tiles is None:
        raise InfeasibleGrid(f"no tile layout for lmax={lmax} k={k} margin={thr}")
    g = Grid(lmax=lmax, k=k, nrings=nrings, nbands_hemi=n, theta=theta,
             sin_theta=s, cos_theta=c, weight=w, alpha=alpha, tiles_north=tiles)
    pix = 0
    tile = 0
    for i in range(n):
        north = [i * k + r for r in range(k)]
        south = [nrings - 1 - (i * k + k - 1) + r for r in range(k)]   # theta increasing
        for rings in (north, south):
            g.band_tiles.append(tiles[i])
            g.band_alpha.append(alpha[i])
            g.band_rings.append(rings)
            g.band_pix0.append(pix)
            g.band_tile0.append(tile)
            pix += tiles[i] * k * k
            tile += tiles[i]
    g.npix = pix
    g.ntiles = tile
    return g
