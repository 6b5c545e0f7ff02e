// Host check of the class-grid dispatch tables (geometry only, no device):
// for grids of several sizes, the two-hop pattern and a two-grid pair, each
// table holds every member tile exactly once.  Below 32 tiles per CU it is all
// tiles largest first; above, plus empty slots: slot 8 i + x is
// XCD x's i-th tile; XCD x runs the x-th of 8 contiguous class-order ranges of
// equal count (the first n mod 8 one longer); each range runs in class order
// but for its smallest tiles by (nterms + 1) x groups, the fewest that hold 15%
// of its work, which run last, largest first; empty slots only at the ends.
// Prints "dispatch_table_check OK".
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../paper_1504_04653_amd/csrc/geometry.hpp"

using namespace sympix;

static int failures = 0;

#define CHECK(cond)                                                                           \
    do {                                                                                      \
        if (!(cond)) {                                                                        \
            std::fprintf(stderr, "%s: check failed at line %d: %s\n", what, __LINE__, #cond); \
            ++failures;                                                                       \
        }                                                                                     \
    } while (0)

static void check_table(const char *what, const ClassTables &ct, const std::vector<int32_t> &tiles,
                        const std::vector<int32_t> &table) {
    const int64_t n = (int64_t)tiles.size() / 4;
    std::map<std::array<int32_t, 4>, int64_t> pos;   // tile -> index in class order
    for (int64_t i = 0; i < n; ++i) {
        std::array<int32_t, 4> t{tiles[4 * i], tiles[4 * i + 1], tiles[4 * i + 2], tiles[4 * i + 3]};
        CHECK(t[2] > 0);
        CHECK(pos.emplace(t, i).second);
    }
    auto cost = [&](int64_t i) { return (int64_t)(ct.classes[tiles[4 * i]].nterms + 1) * tiles[4 * i + 2]; };
    const int64_t slots = (int64_t)table.size() / 4;
    std::vector<int> seen(n, 0);
    if (n < 32 * 256) {                  // short launches: every tile once, largest first, ties in class order
        CHECK(slots == n);
        int64_t prev = -1;
        for (int64_t s = 0; s < slots; ++s) {
            std::array<int32_t, 4> t{table[4 * s], table[4 * s + 1], table[4 * s + 2], table[4 * s + 3]};
            auto it = pos.find(t);
            CHECK(it != pos.end());
            if (it == pos.end()) return;
            const int64_t i = it->second;
            ++seen[i];
            if (prev >= 0) CHECK(cost(prev) > cost(i) || (cost(prev) == cost(i) && prev < i));
            prev = i;
        }
        for (int64_t i = 0; i < n; ++i) CHECK(seen[i] == 1);
        return;
    }
    CHECK(table.size() % 32 == 0);
    const int64_t per = n / 8, rem = n % 8;
    CHECK(slots == 8 * (per + (rem > 0)));
    int64_t next = 0;                    // first class-order index of the next range
    for (int x = 0; x < 8; ++x) {
        std::vector<int64_t> idx;
        bool pad = false;
        for (int64_t s = x; s < slots; s += 8) {
            std::array<int32_t, 4> t{table[4 * s], table[4 * s + 1], table[4 * s + 2], table[4 * s + 3]};
            if (t[2] == 0) {
                CHECK(t[0] == 0 && t[1] == 0 && t[3] == 0);
                pad = true;
                continue;
            }
            CHECK(!pad);                 // empty slots only after the range's tiles
            auto it = pos.find(t);
            CHECK(it != pos.end());
            if (it == pos.end()) return;
            idx.push_back(it->second);
            ++seen[it->second];
        }
        const int64_t count = per + (x < rem);
        CHECK((int64_t)idx.size() == count);
        // the expected tail: tiles by (cost, index) ascending while they hold under 15% of the work
        std::vector<int64_t> rng(count);
        int64_t work = 0;
        for (int64_t j = 0; j < count; ++j) {
            rng[j] = next + j;
            work += cost(rng[j]);
        }
        std::vector<int64_t> byc = rng;
        std::sort(byc.begin(), byc.end(), [&](int64_t u, int64_t v) {
            return cost(u) != cost(v) ? cost(u) < cost(v) : u < v;
        });
        std::vector<char> in_tail(n, 0);
        int64_t acc = 0, ntail = 0;
        while (ntail < count && 100 * acc < 15 * work) {
            in_tail[byc[ntail]] = 1;
            acc += cost(byc[ntail++]);
        }
        if (count > 0 && work > 0) {
            CHECK(100 * acc >= 15 * work);
        }
        std::vector<int64_t> expect;
        for (int64_t i : rng)
            if (!in_tail[i]) expect.push_back(i);
        std::vector<int64_t> t(byc.begin(), byc.begin() + ntail);
        std::sort(t.begin(), t.end(), [&](int64_t u, int64_t v) {
            return cost(u) != cost(v) ? cost(u) > cost(v) : u < v;
        });
        expect.insert(expect.end(), t.begin(), t.end());
        CHECK(idx == expect);
        for (int64_t i : t)              // the tail holds the range's smallest tiles
            for (int64_t j : rng)
                if (!in_tail[j]) CHECK(cost(i) <= cost(j));
        next += count;
    }
    CHECK(next == n);
    for (int64_t i = 0; i < n; ++i) CHECK(seen[i] == 1);
}

static void check_classes(const char *what, const ClassTables &ct) {
    check_table(what, ct, ct.mtiles, ct.gtiles);
    check_table(what, ct, ct.mtiles32, ct.gtiles32);
}

int main() {
    const int sizes[][2] = {{1, 8}, {7, 8}, {16, 8}, {64, 8}, {256, 8}, {512, 8}, {1500, 8}, {2048, 8}, {3000, 8},
                            {40, 4}, {30, 3}};
    int64_t long_tables = 0;
    for (auto &sz : sizes) {
        Geometry g;
        std::string err;
        const std::string what = "grid lmax " + std::to_string(sz[0]) + " k " + std::to_string(sz[1]);
        if (build_geometry(sz[0], sz[1], std::nan(""), g, err) != 0) {
            std::fprintf(stderr, "%s: %s\n", what.c_str(), err.c_str());
            return 1;
        }
        check_classes(what.c_str(), g.cls);
        {   // convolution chunks: every tile in exactly one chunk of its band; workgroups in
            // dispatch order take them largest first
            const char *w = what.c_str();
            const int64_t nc = (int64_t)g.conv_chunks.size() / 4, per = nc / 8, rem = nc % 8;
            std::vector<int> covered(g.ntiles, 0);
            int64_t prev = -1;
            for (int64_t wg = 0; wg < nc; ++wg) {
                const int64_t x = wg & 7, i = wg >> 3, ch = x * per + std::min(x, rem) + i;
                const int32_t *c = &g.conv_chunks[4 * ch];
                for (int32_t t = 0; t < c[1]; ++t) ++covered[c[0] + t];
                if (prev >= 0) {
                    const char *what = w;
                    CHECK(c[3] <= prev);
                }
                prev = c[3];
            }
            const char *what = w;
            for (int64_t J = 0; J < g.ntiles; ++J) CHECK(covered[J] == 1);
        }
        long_tables += (g.cls.mtiles.size() / 4 >= 32 * 256) + (g.cls.mtiles32.size() / 4 >= 32 * 256);
        if (sz[0] == 64 || sz[0] == 256) {
            Pattern p;
            if (build_two_hop(g, p, err) != 0) return 1;
            check_classes((what + " two-hop").c_str(), p.cls);
            Geometry g2;
            if (build_geometry(2 * sz[0], sz[1], std::nan(""), g2, err) != 0) return 1;
            CrossGeometry x;
            if (build_cross(g2, g, x, err) != 0) return 1;
            check_classes((what + " cross").c_str(), x.cls);
        }
    }
    if (long_tables < 2) {
        std::fprintf(stderr, "dispatch_table_check: the per-XCD layout was not exercised\n");
        ++failures;
    }
    if (failures) {
        std::fprintf(stderr, "dispatch_table_check: %d failed checks\n", failures);
        return 1;
    }
    std::printf("dispatch_table_check OK\n");
    return 0;
}
