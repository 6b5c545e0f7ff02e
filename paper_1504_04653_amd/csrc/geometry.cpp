// Host-side SymPix geometry (Section 2 of Seljebotn & Eriksen, Fig. 3).
//
// Compiled with -ffp-contract=off: the ring latitudes feed integer decisions
// (the polar cut of Eq. 3), so every floating-point expression is evaluated
// exactly as written, one rounding per operation.
#include "geometry.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <new>
#include <tuple>
#include <unordered_map>

namespace sympix {
namespace {

constexpr double kPi = 3.141592653589793;

// P_n(1-y) and P_{n-1}(1-y) for n >= 1, by the Legendre recurrence written in
// y = 1 - x with D_l = P_l - P_{l-1}: D_1 = -y,
// (l+1) D_{l+1} = l D_l - (2l+1) y P_l, P_{l+1} = P_l + D_{l+1}.
void legendre_pair_y(int n, double y, double &pn, double &pn1) {
    double p_prev = 1.0;
    double d = -y;
    double p = p_prev + d;
    for (int l = 1; l < n; ++l) {
        d = ((double)l * d - (double)(2 * l + 1) * y * p) / (double)(l + 1);
        p_prev = p;
        p = p + d;
    }
    pn = p;
    pn1 = p_prev;
}

double half_angle_y(double th) {
    double s = std::sin(0.5 * th);
    return 2.0 * (s * s);
}

double newton_step(int n, double th) {
    double y = half_angle_y(th);
    double x = std::cos(th);
    double pn, pn1;
    legendre_pair_y(n, y, pn, pn1);
    return pn * std::sin(th) / ((double)n * (pn1 - x * pn));
}

// Gauss-Legendre colatitudes and weights (Section 2.1, Eq. 2): Newton in
// theta on P_N(cos theta) for the northern half, mirrored to the south.
void gauss_legendre(int n, Geometry &g) {
    const int half = n / 2;
    std::vector<double> th(half);
    for (int j = 0; j < half; ++j)
        th[j] = kPi * (4.0 * (double)j + 3.0) / (4.0 * (double)n + 2.0);
    const double eps = std::numeric_limits<double>::epsilon();
    std::vector<double> step(half);
    for (int it = 0; it < 100; ++it) {
        bool done = true;
        for (int j = 0; j < half; ++j) step[j] = newton_step(n, th[j]);
        for (int j = 0; j < half; ++j) {
            th[j] = th[j] + step[j];
            if (!(std::fabs(step[j]) <= 4.0 * eps * th[j])) done = false;
        }
        if (done) break;
    }
    for (int j = 0; j < half; ++j) th[j] = th[j] + newton_step(n, th[j]);

    g.theta.assign(n, 0.0);
    g.sin_theta.assign(n, 0.0);
    g.cos_theta.assign(n, 0.0);
    g.weight.assign(n, 0.0);
    for (int j = 0; j < half; ++j) {
        double pn, pn1;
        legendre_pair_y(n, half_angle_y(th[j]), pn, pn1);
        double s = std::sin(th[j]);
        double c = std::cos(th[j]);
        double np1 = (double)n * pn1;
        double w = 2.0 * s * s / (np1 * np1);
        g.theta[j] = th[j];
        g.sin_theta[j] = s;
        g.cos_theta[j] = c;
        g.weight[j] = w;
        g.theta[n - 1 - j] = kPi - th[j];
        g.sin_theta[n - 1 - j] = s;
        g.cos_theta[n - 1 - j] = -c;
        g.weight[n - 1 - j] = w;
    }
}

// Smallest m in [0, lmax] with sqrt(m^2 - 2 m cos(theta)) - lmax sin(theta) > thr
// (Eq. 3); a negative radicand does not satisfy it.  -1 if none does.
int min_m_eq3(int lmax, double s, double c, double thr) {
    for (int m = 0; m <= lmax; ++m) {
        double rad = (double)((int64_t)m * m) - 2.0 * (double)m * c;
        if (rad < 0.0) continue;
        if (std::sqrt(rad) - (double)lmax * s > thr) return m;
    }
    return -1;
}

bool five_smooth(int64_t t) {
    for (int p : {2, 3, 5})
        while (t % p == 0) t /= p;
    return t == 1;
}

// Fig. 3: minimise sum (T_i - alpha_i)^2 with T_0 the smallest 5-smooth number
// >= alpha_0, T_i / T_{i-1} in {3, 2, 1, 4/3, 5/4, 6/5} (Eq. 5), alpha_i <= T_i
// <= 3 alpha_i, and a change only after a band that did not change (band 1 is
// exempt).  Ties: t_prev ascending, ratios in the listed order, strict <, and
// the final argmin takes the smallest t.  Returns false if infeasible.
bool tile_programme(const std::vector<int32_t> &alpha, std::vector<int32_t> &tiles) {
    static const int ratio[6][2] = {{3, 1}, {2, 1}, {1, 1}, {4, 3}, {5, 4}, {6, 5}};
    const int n = (int)alpha.size();
    int64_t t0 = std::max<int64_t>(alpha[0], 1);
    while (!five_smooth(t0)) ++t0;
    std::vector<std::map<int64_t, int64_t>> C(n);
    std::vector<std::map<int64_t, int64_t>> P(n);
    C[0][t0] = (t0 - alpha[0]) * (t0 - alpha[0]);
    P[0][t0] = -1;
    for (int i = 1; i < n; ++i) {
        const int64_t a = alpha[i];
        for (const auto &cp : C[i - 1]) {
            const int64_t tp = cp.first;
            const int64_t prev_ptr = P[i - 1][tp];
            for (const auto &r : ratio) {
                if ((r[0] * tp) % r[1]) continue;
                const int64_t t = r[0] * tp / r[1];
                if (t < a || t > 3 * a) continue;
                const bool steady = prev_ptr == tp || r[0] == r[1] || i == 1;
                if (!steady) continue;
                const int64_t cand = cp.second + (a - t) * (a - t);
                auto it = C[i].find(t);
                if (it == C[i].end() || cand < it->second) {
                    C[i][t] = cand;
                    P[i][t] = tp;
                }
            }
        }
    }
    if (C[n - 1].empty()) return false;
    int64_t best = std::numeric_limits<int64_t>::max(), tbest = 0;
    for (const auto &c : C[n - 1])   // ascending t: first minimiser is the smallest t
        if (c.second < best) { best = c.second; tbest = c.first; }
    tiles.assign(n, 0);
    tiles[n - 1] = (int32_t)tbest;
    for (int i = n - 1; i > 0; --i) tiles[i - 1] = (int32_t)P[i][tiles[i]];
    return true;
}

int64_t floor_div(int64_t a, int64_t b) {   // b > 0
    int64_t q = a / b;
    if ((a % b) != 0 && (a < 0)) --q;
    return q;
}

int64_t pos_mod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

// Dispatch table of a launch with one workgroup per member tile.  Workgroup w
// runs on XCD w mod 8, whose CUs take that XCD's workgroups in order as they
// free up.  The tiles, in class order, are cut into 8 contiguous ranges of
// equal count: a class's tiles, which read the same unique blocks, stay on one
// XCD and in its L2, and heavy and light tiles stay mixed, so that MFMA work
// and output stores overlap on every CU.  Each range runs in class order except
// its smallest tiles (by (nterms + 1) x groups, the 1 for the stores) that
// hold kTailPercent of its work: they run last, largest first, and fill the
// CUs that finish early, so that no large tile starts when the rest are done.
// Slot 8 i + x holds the i-th tile of range x; ranges shorter than the first
// end in an empty slot (groups 0).  A launch of fewer than kShortLaunchTiles
// tiles (32 per CU) is too short for that: there the last few tiles of every
// CU set the time, and the table is all tiles largest first (stable).
std::vector<int32_t> xcd_dispatch_table(const std::vector<BlockClass> &classes, const std::vector<int32_t> &tiles) {
    constexpr int kX = 8;
    constexpr int64_t kTailPercent = 15;
    const int64_t n = (int64_t)tiles.size() / 4, per = n / kX, rem = n % kX;
    auto cost = [&](int64_t i) { return (int64_t)(classes[tiles[4 * i]].nterms + 1) * tiles[4 * i + 2]; };
    if (n < kShortLaunchTiles) {
        std::vector<int64_t> order(n);
        for (int64_t i = 0; i < n; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int64_t u, int64_t v) { return cost(u) > cost(v); });
        std::vector<int32_t> out(4 * n);
        for (int64_t i = 0; i < n; ++i) std::copy_n(tiles.begin() + 4 * order[i], 4, out.begin() + 4 * i);
        return out;
    }
    const int64_t len = per + (rem > 0);
    std::vector<int32_t> out(4 * kX * len, 0);
    std::vector<int64_t> order, seq;
    for (int64_t x = 0; x < kX; ++x) {
        const int64_t b = x * per + std::min(x, rem), e = b + per + (x < rem);
        int64_t work = 0;
        order.clear();
        for (int64_t i = b; i < e; ++i) {
            work += cost(i);
            order.push_back(i);
        }
        // the tail: the first tiles of the range ordered by cost, until they hold the share
        std::stable_sort(order.begin(), order.end(), [&](int64_t u, int64_t v) { return cost(u) < cost(v); });
        std::vector<char> tail(e - b, 0);
        int64_t acc = 0, ntail = 0;
        for (; ntail < (int64_t)order.size() && 100 * acc < kTailPercent * work; ++ntail) {
            tail[order[ntail] - b] = 1;
            acc += cost(order[ntail]);
        }
        seq.clear();
        for (int64_t i = b; i < e; ++i)
            if (!tail[i - b]) seq.push_back(i);
        const size_t head = seq.size();
        seq.insert(seq.end(), order.begin(), order.begin() + ntail);
        std::stable_sort(seq.begin() + head, seq.end(), [&](int64_t u, int64_t v) { return cost(u) > cost(v); });
        for (size_t j = 0; j < seq.size(); ++j)
            std::copy_n(tiles.begin() + 4 * seq[j], 4, out.begin() + 4 * (kX * (int64_t)j + x));
    }
    return out;
}

// Block classes of a stored-block pattern: key = the sorted (uid_a, uid_b)
// pairs of a block's terms; member tiles of 64 rows (a tail of at most 48
// members in tiles of 32 and / or 16) and, as a second tile shape, of 32.
void build_classes(const std::vector<int64_t> &term_ptr, const std::vector<Term> &terms, ClassTables &ct) {
    struct VecHash {
        size_t operator()(const std::vector<int32_t> &v) const {
            uint64_t h = 1469598103934665603ull;
            for (int32_t x : v) h = (h ^ (uint32_t)x) * 1099511628211ull;
            return (size_t)h;
        }
    };
    const int64_t nblocks = (int64_t)term_ptr.size() - 1;
    std::unordered_map<std::vector<int32_t>, int32_t, VecHash> index;
    std::vector<std::vector<int32_t>> members;     // per class: block indices
    std::vector<std::vector<int32_t>> tiles_of;    // per class: I per (member, term)
    std::vector<std::vector<int32_t>> keys;
    std::vector<std::tuple<int32_t, int32_t, int32_t>> tt;
    std::vector<int32_t> key;
    for (int64_t n = 0; n < nblocks; ++n) {
        tt.clear();
        for (int64_t t = term_ptr[n]; t < term_ptr[n + 1]; ++t)
            tt.emplace_back(terms[t].uid_a, terms[t].uid_b, terms[t].tile);
        std::sort(tt.begin(), tt.end());
        key.clear();
        for (auto &x : tt) {
            key.push_back(std::get<0>(x));
            key.push_back(std::get<1>(x));
        }
        auto it = index.find(key);
        int32_t c;
        if (it == index.end()) {
            c = (int32_t)keys.size();
            index.emplace(key, c);
            keys.push_back(key);
            members.emplace_back();
            tiles_of.emplace_back();
        } else {
            c = it->second;
        }
        members[c].push_back((int32_t)n);
        for (auto &x : tt) tiles_of[c].push_back(std::get<2>(x));
    }
    for (size_t c = 0; c < keys.size(); ++c) {
        BlockClass bc;
        bc.nterms = (int32_t)(keys[c].size() / 2);
        ct.max_class_terms = std::max(ct.max_class_terms, bc.nterms);
        bc.nblocks = (int32_t)members[c].size();
        bc.term0 = (int32_t)(ct.class_terms.size() / 2);
        bc.blk0 = (int32_t)ct.class_blk.size();
        bc.itab0 = (int64_t)ct.class_itab.size();
        bc.sym = 1;
        for (size_t q = 0; q + 1 < keys[c].size(); q += 2) bc.sym &= keys[c][q] == keys[c][q + 1] ? 1 : 0;
        bc.pad = 0;
        ct.class_terms.insert(ct.class_terms.end(), keys[c].begin(), keys[c].end());
        ct.class_blk.insert(ct.class_blk.end(), members[c].begin(), members[c].end());
        ct.class_itab.insert(ct.class_itab.end(), tiles_of[c].begin(), tiles_of[c].end());
        auto tile = [&](int32_t m0, int32_t groups) {
            ct.mtiles.insert(ct.mtiles.end(), {(int32_t)c, m0, groups, 0});
        };
        int32_t m0 = 0;
        for (; bc.nblocks - m0 > 48; m0 += 64) tile(m0, 4);
        const int32_t r = bc.nblocks - m0;
        if (r > 32) {
            tile(m0, 2);
            tile(m0 + 32, 1);
        } else if (r > 16) {
            tile(m0, 2);
        } else if (r > 0) {
            tile(m0, 1);
        }
        int32_t mb = 0;
        for (; bc.nblocks - mb > 16; mb += 32) ct.mtiles32.insert(ct.mtiles32.end(), {(int32_t)c, mb, 2, 0});
        if (bc.nblocks - mb > 0) ct.mtiles32.insert(ct.mtiles32.end(), {(int32_t)c, mb, 1, 0});
        ct.classes.push_back(bc);
    }
    ct.gtiles = xcd_dispatch_table(ct.classes, ct.mtiles);
    ct.gtiles32 = xcd_dispatch_table(ct.classes, ct.mtiles32);
}

}  // namespace

// Largest y = 1 - cos(gamma) over every pair of a set of blocks: per block
// the largest |phi offset| over the k x k column pairs, then every ring pair.
// Rows on grid gi (tile I), columns on grid gj (tile J).
static double blocks_y_max(const Geometry &gi, const Geometry &gj, const std::vector<int32_t> &rep_i,
                           const std::vector<int32_t> &rep_j) {
    const int k = gj.k;
    double ymax = 0.0;
    for (size_t u = 0; u < rep_i.size(); ++u) {
        const int64_t I = rep_i[u], J = rep_j[u];
        const int bI = gi.tile_band[I], bJ = gj.tile_band[J];
        const int64_t nI = (int64_t)k * gi.band_tiles[bI], nJ = (int64_t)k * gj.band_tiles[bJ];
        const int64_t pI0 = (I - gi.band_tile0[bI]) * k, pJ0 = (J - gj.band_tile0[bJ]) * k;
        const int64_t M = nI * nJ;
        int64_t nmax = 0;
        for (int c = 0; c < k; ++c)
            for (int c2 = 0; c2 < k; ++c2) {
                int64_t N = pos_mod((2 * (pJ0 + c2) + 1) * nI - (2 * (pI0 + c) + 1) * nJ, 2 * M);
                if (N > M) N -= 2 * M;
                nmax = std::max(nmax, N < 0 ? -N : N);
            }
        const double sh = std::sin(0.5 * (kPi * (double)nmax / (double)M));
        const double hmax = sh * sh;
        for (int r = 0; r < k; ++r)
            for (int r2 = 0; r2 < k; ++r2) {
                const int j1 = gi.band_ring0[bI] + r, j2 = gj.band_ring0[bJ] + r2;
                const double sd = std::sin(0.5 * (gi.theta[j1] - gj.theta[j2]));
                const double y = 2.0 * (sd * sd + gi.sin_theta[j1] * gj.sin_theta[j2] * hmax);
                ymax = std::max(ymax, y);
            }
    }
    return ymax;
}

int build_geometry(int32_t lmax, int32_t k, double margin, Geometry &g, std::string &err) {
    try {
        if (lmax < 1 || k < 1 || k > 64 || lmax > 100000) {
            err = "lmax must be in [1, 100000] and k in [1, 64]";
            return -1;
        }
        g = Geometry();
        g.lmax = lmax;
        g.k = k;
        g.nrings = (int32_t)(((int64_t)lmax + 1 + 2 * k - 1) / (2 * k) * (2 * k));
        g.nbands_hemi = g.nrings / (2 * k);
        g.margin = std::isnan(margin) ? std::max(100.0, 0.01 * (double)lmax) : margin;
        if (!std::isfinite(g.margin)) {
            err = "polar_margin must be finite (or NaN for the default)";
            return -1;
        }
        const int n = g.nbands_hemi;
        gauss_legendre(g.nrings, g);

        // alpha_i at the pole-most ring of each northern band (Fig. 3)
        g.alpha_north.resize(n);
        for (int i = 0; i < n; ++i) {
            const int j = i * k;
            int m = min_m_eq3(lmax, g.sin_theta[j], g.cos_theta[j], g.margin);
            if (m < 0) m = lmax;
            g.alpha_north[i] = (int32_t)((2 * (int64_t)m + 1 + k - 1) / k);
        }
        if (!tile_programme(g.alpha_north, g.tiles_north)) {
            err = "no tile layout satisfies the rules of Fig. 3 for this lmax, k and margin";
            return -2;
        }

        // bands in storage order N0, S0, N1, S1, ... (Section 2.4), rings by increasing theta
        int64_t tile = 0;
        for (int i = 0; i < n; ++i) {
            for (int south = 0; south < 2; ++south) {
                g.band_tiles.push_back(g.tiles_north[i]);
                g.band_alpha.push_back(g.alpha_north[i]);
                g.band_ring0.push_back(south ? g.nrings - i * k - k : i * k);
                g.band_tile0.push_back(tile);
                tile += g.tiles_north[i];
            }
        }
        g.ntiles = tile;
        g.npix = tile * (int64_t)k * k;
        const int nb = 2 * n;
        g.tile_band.resize(g.ntiles);
        for (int b = 0; b < nb; ++b)
            for (int64_t t = 0; t < g.band_tiles[b]; ++t) g.tile_band[g.band_tile0[b] + t] = b;
        g.ring_npix.assign(g.nrings, 0);
        g.ring_first_pix.assign(g.nrings, 0);
        for (int b = 0; b < nb; ++b)
            for (int r = 0; r < k; ++r) {
                g.ring_npix[g.band_ring0[b] + r] = k * g.band_tiles[b];
                g.ring_first_pix[g.band_ring0[b] + r] = g.band_tile0[b] * k * k + r;
            }

        // tile adjacency (Section 2.2): same band t-1, t, t+1 mod T; neighbouring
        // bands by closed phi-interval intersection, in integers scaled by T T'
        g.adj_ptr.assign(g.ntiles + 1, 0);
        std::vector<int32_t> row;
        for (int64_t I = 0; I < g.ntiles; ++I) {
            const int b = g.tile_band[I];
            const int64_t T = g.band_tiles[b];
            const int64_t t = I - g.band_tile0[b];
            row.clear();
            for (int d = -1; d <= 1; ++d) row.push_back((int32_t)(g.band_tile0[b] + pos_mod(t + d, T)));
            const int i = b / 2, south = b % 2;
            int nbrs[2], nn = 0;
            if (i > 0) nbrs[nn++] = 2 * (i - 1) + south;
            if (i < n - 1) nbrs[nn++] = 2 * (i + 1) + south;
            else nbrs[nn++] = 2 * i + (1 - south);
            for (int q = 0; q < nn; ++q) {
                const int b2 = nbrs[q];
                const int64_t T2 = g.band_tiles[b2];
                const int64_t M = T * T2;
                const int64_t lo1 = t * T2, hi1 = (t + 1) * T2;
                int64_t u0 = 0, u1 = T2 - 1;
                if (T2 > 8) { u0 = floor_div(t * T2, T) - 1; u1 = floor_div((t + 1) * T2, T) + 1; }
                for (int64_t u = u0; u <= u1; ++u) {
                    const int64_t t2 = pos_mod(u, T2);
                    const int64_t lo2 = t2 * T, hi2 = (t2 + 1) * T;
                    for (int64_t shift : {-M, (int64_t)0, M}) {
                        if (lo1 <= hi2 + shift && lo2 + shift <= hi1) {
                            row.push_back((int32_t)(g.band_tile0[b2] + t2));
                            break;
                        }
                    }
                }
            }
            std::sort(row.begin(), row.end());
            row.erase(std::unique(row.begin(), row.end()), row.end());
            g.adj_col.insert(g.adj_col.end(), row.begin(), row.end());
            g.adj_ptr[I + 1] = (int64_t)g.adj_col.size();
        }

        // symmetry keys (band_I, band_J, (t_J T_I - t_I T_J) mod T_I T_J)
        std::map<std::tuple<int32_t, int32_t, int64_t>, int32_t> keys;
        g.adj_uid.resize(g.adj_col.size());
        for (int64_t I = 0; I < g.ntiles; ++I) {
            const int bI = g.tile_band[I];
            const int64_t TI = g.band_tiles[bI], tI = I - g.band_tile0[bI];
            for (int64_t e = g.adj_ptr[I]; e < g.adj_ptr[I + 1]; ++e) {
                const int64_t J = g.adj_col[e];
                const int bJ = g.tile_band[J];
                const int64_t TJ = g.band_tiles[bJ], tJ = J - g.band_tile0[bJ];
                const int64_t delta = pos_mod(tJ * TI - tI * TJ, TI * TJ);
                auto key = std::make_tuple((int32_t)bI, (int32_t)bJ, delta);
                auto it = keys.find(key);
                int32_t uid;
                if (it == keys.end()) {
                    uid = (int32_t)g.key_delta.size();
                    keys.emplace(key, uid);
                    g.key_band_i.push_back(bI);
                    g.key_band_j.push_back(bJ);
                    g.key_delta.push_back(delta);
                    g.rep_i.push_back((int32_t)I);
                    g.rep_j.push_back((int32_t)J);
                } else {
                    uid = it->second;
                }
                g.adj_uid[e] = uid;
            }
        }

        auto uid_of = [&](int64_t I, int64_t J) -> int32_t {
            auto first = g.adj_col.begin() + g.adj_ptr[I], last = g.adj_col.begin() + g.adj_ptr[I + 1];
            auto it = std::lower_bound(first, last, (int32_t)J);
            return g.adj_uid[it - g.adj_col.begin()];
        };

        // stored blocks (J, K >= J) and their contraction terms I in nbr(J) & nbr(K)
        g.blk_ptr.assign(g.ntiles + 1, 0);
        g.term_ptr.push_back(0);
        for (int64_t J = 0; J < g.ntiles; ++J) {
            for (int64_t e = g.adj_ptr[J]; e < g.adj_ptr[J + 1]; ++e) {
                const int64_t K = g.adj_col[e];
                if (K < J) continue;
                g.blk_col.push_back((int32_t)K);
                g.blk_uid.push_back(g.adj_uid[e]);
                auto a = g.adj_col.begin() + g.adj_ptr[J], ae = g.adj_col.begin() + g.adj_ptr[J + 1];
                auto b = g.adj_col.begin() + g.adj_ptr[K], be = g.adj_col.begin() + g.adj_ptr[K + 1];
                while (a != ae && b != be) {
                    if (*a < *b) ++a;
                    else if (*b < *a) ++b;
                    else {
                        const int64_t I = *a;
                        g.terms.push_back(Term{uid_of(I, J), uid_of(I, K), (int32_t)I, 0});
                        ++a;
                        ++b;
                    }
                }
                g.term_ptr.push_back((int64_t)g.terms.size());
            }
            g.blk_ptr[J + 1] = (int64_t)g.blk_col.size();
        }

        // D-hat expansion list: stored blocks grouped by unique block, in work
        // items of at most 64 blocks {uid, first, count, 0}
        {
            std::vector<int32_t> cnt(g.nunique() + 1, 0);
            for (int32_t u : g.blk_uid) ++cnt[u + 1];
            for (int64_t u = 0; u < g.nunique(); ++u) cnt[u + 1] += cnt[u];
            g.exp_blk.assign(g.nblocks(), 0);
            std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
            for (int64_t n = 0; n < g.nblocks(); ++n) g.exp_blk[pos[g.blk_uid[n]]++] = (int32_t)n;
            for (int64_t u = 0; u < g.nunique(); ++u)
                for (int32_t f = cnt[u]; f < cnt[u + 1]; f += 64)
                    g.exp_items.insert(g.exp_items.end(), {(int32_t)u, f, std::min(64, cnt[u + 1] - f), 0});
        }

        // convolution chunks: kConvTiles consecutive tiles of one band; a slot per unique
        // block used, listing the input tile of every output tile (a tile uses a
        // unique block with at most one neighbour, else a further slot is made)
        {
            const int nb = (int)g.band_tiles.size();
            for (int b = 0; b < nb; ++b) {
                const int32_t T = g.band_tiles[b];
                for (int32_t c0 = 0; c0 < T; c0 += kConvTiles) {
                    const int32_t J0 = (int32_t)g.band_tile0[b] + c0, n = std::min(kConvTiles, T - c0);
                    const int32_t slot0 = (int32_t)(g.conv_slots.size() / (1 + kConvTiles));
                    std::vector<int32_t> slots;          // 1 + kConvTiles per slot
                    for (int32_t j = 0; j < n; ++j) {
                        const int64_t J = J0 + j;
                        for (int64_t e = g.adj_ptr[J]; e < g.adj_ptr[J + 1]; ++e) {
                            const int32_t u = g.adj_uid[e], K = g.adj_col[e];
                            size_t sidx = 0;
                            for (; sidx < slots.size(); sidx += 1 + kConvTiles)
                                if (slots[sidx] == u && slots[sidx + 1 + j] < 0) break;
                            if (sidx == slots.size()) {
                                slots.push_back(u);
                                slots.insert(slots.end(), kConvTiles, -1);
                            }
                            slots[sidx + 1 + j] = K;
                        }
                    }
                    g.conv_slots.insert(g.conv_slots.end(), slots.begin(), slots.end());
                    g.conv_chunks.insert(g.conv_chunks.end(), {J0, n, slot0, (int32_t)(slots.size() / (1 + kConvTiles))});
                }
            }
            // The launch gives workgroup w the chunk (w mod 8) per + min(w mod 8, rem) + w / 8
            // (an XCD-contiguous map); place the chunks so that the workgroups, dispatched in
            // order, take them largest first (slots, stable): the last chunks of every CU are
            // then the small ones
            const int64_t nc = (int64_t)g.conv_chunks.size() / 4, per = nc / 8, rem = nc % 8;
            std::vector<int64_t> order(nc);
            for (int64_t i = 0; i < nc; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(),
                             [&](int64_t a, int64_t b) { return g.conv_chunks[4 * a + 3] > g.conv_chunks[4 * b + 3]; });
            std::vector<int32_t> placed(g.conv_chunks.size());
            for (int64_t w = 0; w < nc; ++w) {
                const int64_t x = w & 7, i = w >> 3, ch = x * per + std::min(x, rem) + i;
                std::copy_n(g.conv_chunks.begin() + 4 * order[w], 4, placed.begin() + 4 * ch);
            }
            g.conv_chunks.swap(placed);
        }

        build_classes(g.term_ptr, g.terms, g.cls);

        g.y_pattern_max = blocks_y_max(g, g, g.rep_i, g.rep_j);
        return 0;
    } catch (const std::bad_alloc &) {
        err = "host allocation failed while building the grid";
        return -3;
    }
}


int build_two_hop(const Geometry &g, Pattern &p, std::string &err) {
    try {
        p = Pattern();
        auto uid_of = [&](int64_t I, int64_t J) -> int32_t {
            auto first = g.adj_col.begin() + g.adj_ptr[I], last = g.adj_col.begin() + g.adj_ptr[I + 1];
            auto it = std::lower_bound(first, last, (int32_t)J);
            return g.adj_uid[it - g.adj_col.begin()];
        };
        // blocks (J, K >= J) with nbr(J) & nbr(K) non-empty, K ascending; terms
        // I in nbr(J) & nbr(K), ascending
        p.blk_ptr.assign(g.ntiles + 1, 0);
        p.term_ptr.push_back(0);
        std::vector<int32_t> ks;
        for (int64_t J = 0; J < g.ntiles; ++J) {
            ks.clear();
            for (int64_t e = g.adj_ptr[J]; e < g.adj_ptr[J + 1]; ++e) {
                const int64_t I = g.adj_col[e];
                for (int64_t f = g.adj_ptr[I]; f < g.adj_ptr[I + 1]; ++f)
                    if (g.adj_col[f] >= J) ks.push_back(g.adj_col[f]);
            }
            std::sort(ks.begin(), ks.end());
            ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
            for (int32_t K : ks) {
                p.blk_col.push_back(K);
                auto a = g.adj_col.begin() + g.adj_ptr[J], ae = g.adj_col.begin() + g.adj_ptr[J + 1];
                auto b = g.adj_col.begin() + g.adj_ptr[K], be = g.adj_col.begin() + g.adj_ptr[K + 1];
                while (a != ae && b != be) {
                    if (*a < *b) ++a;
                    else if (*b < *a) ++b;
                    else {
                        const int64_t I = *a;
                        p.terms.push_back(Term{uid_of(I, J), uid_of(I, K), (int32_t)I, 0});
                        ++a;
                        ++b;
                    }
                }
                p.term_ptr.push_back((int64_t)p.terms.size());
            }
            p.blk_ptr[J + 1] = (int64_t)p.blk_col.size();
        }
        build_classes(p.term_ptr, p.terms, p.cls);
        return 0;
    } catch (const std::bad_alloc &) {
        err = "host allocation failed building the two-hop pattern";
        return -3;
    }
}

int build_cross(const Geometry &g2, const Geometry &g1, CrossGeometry &x, std::string &err) {
    try {
        x = CrossGeometry();
        if (g1.k != g2.k) {
            err = "the two grids must have the same tile size k";
            return -6;
        }
        x.lmax_eff = std::min(g1.lmax, g2.lmax);
        const int64_t k = g1.k, R1 = g1.nrings;
        // the tile of g1 holding the centre of every tile of g2: colatitude
        // (lo + hi) / (2 R2) pi, longitude (2t + 1) / (2T) turn; half-open
        // band ranges [ik, (i+1)k) / R1 north, [R1 - (i+1)k, R1 - ik) / R1 south
        x.container.resize(g2.ntiles);
        for (size_t b = 0; b < g2.band_tiles.size(); ++b) {
            const int64_t i2 = (int64_t)b / 2, south2 = (int64_t)b % 2, R2 = g2.nrings;
            const int64_t lo = south2 ? R2 - (i2 + 1) * k : i2 * k, hi = lo + k;
            const int64_t th_num = lo + hi, th_den = 2 * R2;
            const int64_t xs = th_num * R1;                 // theta R1 = xs / th_den
            int b1;
            if (2 * th_num < th_den) {
                b1 = (int)(2 * (xs / (th_den * k)));
            } else {
                const int64_t ys = R1 * th_den - xs;        // (1 - theta) R1 th_den > 0
                b1 = (int)(2 * ((ys + th_den * k - 1) / (th_den * k) - 1) + 1);
            }
            const int64_t T2 = g2.band_tiles[b], T1 = g1.band_tiles[b1];
            for (int64_t t = 0; t < T2; ++t)
                x.container[g2.band_tile0[b] + t] = (int32_t)(g1.band_tile0[b1] + ((2 * t + 1) * T1) / (2 * T2));
        }
        // adjacency rows: the g1 neighbours of each tile's container; keys in
        // the one-grid order (I ascending, then J ascending)
        std::map<std::tuple<int32_t, int32_t, int64_t>, int32_t> keys;
        x.adj_ptr.assign(g2.ntiles + 1, 0);
        for (int64_t I = 0; I < g2.ntiles; ++I) {
            const int64_t C = x.container[I];
            const int bI = g2.tile_band[I];
            const int64_t TI = g2.band_tiles[bI], tI = I - g2.band_tile0[bI];
            for (int64_t e = g1.adj_ptr[C]; e < g1.adj_ptr[C + 1]; ++e) {
                const int64_t J = g1.adj_col[e];
                const int bJ = g1.tile_band[J];
                const int64_t TJ = g1.band_tiles[bJ], tJ = J - g1.band_tile0[bJ];
                const int64_t delta = pos_mod(tJ * TI - tI * TJ, TI * TJ);
                auto key = std::make_tuple((int32_t)bI, (int32_t)bJ, delta);
                auto it = keys.find(key);
                int32_t uid;
                if (it == keys.end()) {
                    uid = (int32_t)x.key_delta.size();
                    keys.emplace(key, uid);
                    x.key_band_i.push_back(bI);
                    x.key_band_j.push_back(bJ);
                    x.key_delta.push_back(delta);
                    x.rep_i.push_back((int32_t)I);
                    x.rep_j.push_back((int32_t)J);
                } else {
                    uid = it->second;
                }
                x.adj_col.push_back((int32_t)J);
                x.adj_uid.push_back(uid);
            }
            x.adj_ptr[I + 1] = (int64_t)x.adj_col.size();
        }
        // transpose: the tiles of g2 neighbouring each tile of g1, ascending
        x.nbr_ptr.assign(g1.ntiles + 1, 0);
        for (int32_t J : x.adj_col) ++x.nbr_ptr[J + 1];
        for (int64_t J = 0; J < g1.ntiles; ++J) x.nbr_ptr[J + 1] += x.nbr_ptr[J];
        x.nbr_col.assign(x.adj_col.size(), 0);
        {
            std::vector<int64_t> pos(x.nbr_ptr.begin(), x.nbr_ptr.end() - 1);
            for (int64_t I = 0; I < g2.ntiles; ++I)
                for (int64_t e = x.adj_ptr[I]; e < x.adj_ptr[I + 1]; ++e) x.nbr_col[pos[x.adj_col[e]]++] = (int32_t)I;
        }
        auto uid_of = [&](int64_t I, int64_t J) -> int32_t {
            auto first = x.adj_col.begin() + x.adj_ptr[I], last = x.adj_col.begin() + x.adj_ptr[I + 1];
            auto it = std::lower_bound(first, last, (int32_t)J);
            return x.adj_uid[it - x.adj_col.begin()];
        };
        // terms of every stored block (J, K) of g1: I in nbr(J) & nbr(K), ascending
        x.term_ptr.push_back(0);
        for (int64_t J = 0; J < g1.ntiles; ++J)
            for (int64_t n = g1.blk_ptr[J]; n < g1.blk_ptr[J + 1]; ++n) {
                const int64_t K = g1.blk_col[n];
                auto a = x.nbr_col.begin() + x.nbr_ptr[J], ae = x.nbr_col.begin() + x.nbr_ptr[J + 1];
                auto b = x.nbr_col.begin() + x.nbr_ptr[K], be = x.nbr_col.begin() + x.nbr_ptr[K + 1];
                while (a != ae && b != be) {
                    if (*a < *b) ++a;
                    else if (*b < *a) ++b;
                    else {
                        const int64_t I = *a;
                        x.terms.push_back(Term{uid_of(I, J), uid_of(I, K), (int32_t)I, 0});
                        ++a;
                        ++b;
                    }
                }
                x.term_ptr.push_back((int64_t)x.terms.size());
            }
        // B-hat output blocks (one per adjacency entry) grouped by unique
        // block, work items of at most 64 {uid, first, count, 0}
        {
            const int64_t nadj = (int64_t)x.adj_col.size();
            std::vector<int64_t> cnt(x.nunique() + 1, 0);
            for (int32_t u : x.adj_uid) ++cnt[u + 1];
            for (int64_t u = 0; u < x.nunique(); ++u) cnt[u + 1] += cnt[u];
            if (nadj >= INT32_MAX) {
                err = "too many B-hat blocks";
                return -5;
            }
            x.exp_blk.assign(nadj, 0);
            std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
            for (int64_t e = 0; e < nadj; ++e) x.exp_blk[pos[x.adj_uid[e]]++] = (int32_t)e;
            for (int64_t u = 0; u < x.nunique(); ++u)
                for (int64_t f = cnt[u]; f < cnt[u + 1]; f += 64)
                    x.exp_items.insert(x.exp_items.end(),
                                       {(int32_t)u, (int32_t)f, (int32_t)std::min<int64_t>(64, cnt[u + 1] - f), 0});
        }
        build_classes(x.term_ptr, x.terms, x.cls);
        x.y_pattern_max = blocks_y_max(g2, g1, x.rep_i, x.rep_j);
        return 0;
    } catch (const std::bad_alloc &) {
        err = "host allocation failed building the two-grid tables";
        return -3;
    }
}

}  // namespace sympix
