// Host-side exercise of the C ABI for a sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code; no device is touched): grid
// creation over many sizes and tile sizes, every layout query into buffers of
// exactly the sizes the dims report, the two-hop pattern, two-grid pairs,
// argument errors, and injected allocation failures.  Prints "abi_host_check
// OK" and exits 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/sympix.h"

static int failures = 0;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static void exercise_grid(int lmax, int k, double margin) {
    sympix_grid *g = nullptr;
    const sympix_status s = sympix_grid_create(lmax, k, margin, &g);
    if (s != SYMPIX_OK) {
        CHECK(g == nullptr);
        return;
    }
    sympix_dims d;
    CHECK(sympix_grid_dims(g, &d) == SYMPIX_OK);
    CHECK(d.npix == d.ntiles * k * k);
    std::vector<double> theta(d.nrings), weight(d.nrings), pth(d.npix), pph(d.npix);
    std::vector<int32_t> npr(d.nrings);
    std::vector<int64_t> first(d.nrings);
    CHECK(sympix_grid_rings(g, theta.data(), weight.data(), npr.data(), first.data()) == SYMPIX_OK);
    double wsum = 0.0;
    for (double w : weight) wsum += w;
    CHECK(std::fabs(wsum - 2.0) < 1e-12);
    std::vector<int32_t> tiles(2 * d.nbands_hemi), alpha(2 * d.nbands_hemi), ring0(2 * d.nbands_hemi);
    CHECK(sympix_grid_bands(g, tiles.data(), alpha.data(), ring0.data()) == SYMPIX_OK);
    CHECK(sympix_grid_pixels(g, pth.data(), pph.data()) == SYMPIX_OK);
    std::vector<int64_t> rp(d.ntiles + 1), brp(d.ntiles + 1);
    std::vector<int32_t> col(d.nadjacency), bcol(d.nblocks), uid(d.nadjacency);
    CHECK(sympix_grid_neighbours(g, rp.data(), col.data()) == SYMPIX_OK);
    CHECK(rp[d.ntiles] == d.nadjacency);
    for (int32_t c : col) CHECK(c >= 0 && c < d.ntiles);
    CHECK(sympix_grid_blocks(g, brp.data(), bcol.data()) == SYMPIX_OK);
    CHECK(brp[d.ntiles] == d.nblocks);
    std::vector<int32_t> kbi(d.nunique), kbj(d.nunique);
    std::vector<int64_t> kde(d.nunique);
    CHECK(sympix_grid_unique(g, uid.data(), kbi.data(), kbj.data(), kde.data()) == SYMPIX_OK);
    for (int32_t u : uid) CHECK(u >= 0 && u < d.nunique);
    int64_t nb2 = 0, nt2 = 0;
    CHECK(sympix_grid_pattern_blocks(g, SYMPIX_PATTERN_TWO_HOP, &nb2, &nt2, nullptr, nullptr) == SYMPIX_OK);
    std::vector<int64_t> rp2(d.ntiles + 1);
    std::vector<int32_t> col2(nb2);
    CHECK(sympix_grid_pattern_blocks(g, SYMPIX_PATTERN_TWO_HOP, nullptr, nullptr, rp2.data(), col2.data()) == SYMPIX_OK);
    CHECK(nb2 >= d.nblocks && nt2 >= d.nterms);
    CHECK(sympix_grid_pattern_blocks(g, 7, &nb2, &nt2, nullptr, nullptr) == SYMPIX_EINVAL);
    // a pair of the grid with itself and with a finer grid of the same k
    sympix_grid *g2 = nullptr;
    if (lmax <= 600 && sympix_grid_create(2 * lmax + 1, k, margin, &g2) == SYMPIX_OK) {
        for (const sympix_grid *aux : {(const sympix_grid *)g, (const sympix_grid *)g2}) {
            sympix_cross *x = nullptr;
            CHECK(sympix_cross_create(aux, g, &x) == SYMPIX_OK);
            sympix_cross_sizes cs;
            CHECK(sympix_cross_dims(x, &cs) == SYMPIX_OK);
            sympix_dims da;
            sympix_grid_dims(aux, &da);
            std::vector<int32_t> cont(da.ntiles), xcol(cs.nadjacency), xuid(cs.nadjacency);
            std::vector<int64_t> xrp(da.ntiles + 1);
            CHECK(sympix_cross_neighbours(x, cont.data(), xrp.data(), xcol.data(), xuid.data()) == SYMPIX_OK);
            for (int32_t c : cont) CHECK(c >= 0 && c < d.ntiles);
            std::vector<int32_t> xbi(cs.nunique), xbj(cs.nunique);
            std::vector<int64_t> xde(cs.nunique);
            CHECK(sympix_cross_unique(x, xbi.data(), xbj.data(), xde.data()) == SYMPIX_OK);
            CHECK(cs.nblocks == d.nblocks);
            sympix_cross_destroy(x);
        }
        sympix_grid_destroy(g2);
    }
    sympix_grid_destroy(g);
}

int main() {
    const double nan = std::nan("");
    const int cases[][2] = {{1, 8}, {7, 8}, {16, 8}, {64, 8}, {100, 8}, {256, 8}, {511, 8}, {20, 2}, {34, 2},
                            {40, 4}, {9, 1}, {30, 3}, {1000, 4}, {1500, 8}};
    for (auto &c : cases) exercise_grid(c[0], c[1], nan);
    exercise_grid(20, 2, 0.0);
    exercise_grid(34, 2, 2.0);
    // argument errors: no handle is returned and nothing leaks
    sympix_grid *g = (sympix_grid *)0x1;
    CHECK(sympix_grid_create(0, 8, nan, &g) == SYMPIX_EINVAL && g == nullptr);
    CHECK(sympix_grid_create(64, 0, nan, &g) == SYMPIX_EINVAL);
    CHECK(sympix_grid_create(64, 65, nan, &g) == SYMPIX_EINVAL);
    CHECK(sympix_grid_create(64, 8, nan, nullptr) == SYMPIX_EINVAL);
    CHECK(sympix_grid_create(64, 8, 0.0, &g) == SYMPIX_EINFEASIBLE && g == nullptr);
    CHECK(sympix_grid_dims(nullptr, nullptr) == SYMPIX_EINVAL);
    CHECK(std::string(sympix_last_error()).size() > 0);
    sympix_grid *a = nullptr, *b = nullptr;
    CHECK(sympix_grid_create(64, 8, nan, &a) == SYMPIX_OK);
    CHECK(sympix_grid_create(40, 4, nan, &b) == SYMPIX_OK);
    sympix_cross *x = (sympix_cross *)0x1;
    CHECK(sympix_cross_create(b, a, &x) == SYMPIX_EUNSUPPORTED && x == nullptr);
    CHECK(sympix_cross_create(nullptr, a, &x) == SYMPIX_EINVAL);
    // injected allocation failures: each point in turn, then none
    for (int n = 1; n <= 3; ++n) {
        setenv("SYMPIX_FAIL_ALLOC", std::to_string(n).c_str(), 1);
        sympix_grid *h = nullptr;
        const sympix_status s = sympix_grid_create(100, 8, nan, &h);
        if (n <= 2) {
            CHECK(s == SYMPIX_ENOMEM && h == nullptr);
        } else {
            CHECK(s == SYMPIX_OK && h != nullptr);
        }
        sympix_grid_destroy(h);
        unsetenv("SYMPIX_FAIL_ALLOC");
    }
    for (int n = 1; n <= 2; ++n) {
        setenv("SYMPIX_FAIL_ALLOC", std::to_string(n).c_str(), 1);
        sympix_cross *h = nullptr;
        CHECK(sympix_cross_create(a, a, &h) == SYMPIX_ENOMEM && h == nullptr);
        unsetenv("SYMPIX_FAIL_ALLOC");
    }
    setenv("SYMPIX_FAIL_ALLOC", "1", 1);
    int64_t nb = 0;
    CHECK(sympix_grid_pattern_blocks(a, SYMPIX_PATTERN_TWO_HOP, &nb, nullptr, nullptr, nullptr) == SYMPIX_ENOMEM);
    unsetenv("SYMPIX_FAIL_ALLOC");
    CHECK(sympix_grid_pattern_blocks(a, SYMPIX_PATTERN_TWO_HOP, &nb, nullptr, nullptr, nullptr) == SYMPIX_OK);
    // transform plans: argument errors and the host allocation are checked
    // before any device call
    sympix_sht *sh = (sympix_sht *)0x1;
    CHECK(sympix_sht_create(nullptr, 10, &sh) == SYMPIX_EINVAL && sh == (sympix_sht *)0x1);
    CHECK(sympix_sht_create(a, -1, &sh) == SYMPIX_EINVAL && sh == nullptr);
    CHECK(sympix_sht_create(a, 5000, &sh) == SYMPIX_EUNSUPPORTED && sh == nullptr);
    setenv("SYMPIX_FAIL_ALLOC", "1", 1);
    CHECK(sympix_sht_create(a, 64, &sh) == SYMPIX_ENOMEM && sh == nullptr);
    unsetenv("SYMPIX_FAIL_ALLOC");
    CHECK(sympix_sht_synthesis(nullptr, nullptr, 0, nullptr, 0, nullptr) == SYMPIX_EINVAL);
    CHECK(sympix_sht_degrade(nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr) == SYMPIX_EINVAL);
    // block-Jacobi factor and solve: argument checks come before any device call
    {
        sympix_dims da;
        CHECK(sympix_grid_dims(a, &da) == SYMPIX_OK);
        const int64_t nb = da.nblocks * 4096, nu = da.ntiles * 4096;
        double *fake = (double *)0x1000;   // never dereferenced: every call below fails its checks
        int32_t *ifake = (int32_t *)0x1000;
        CHECK(sympix_factor_diag(nullptr, fake, nb, nullptr, 0, fake, nu, ifake, da.ntiles, nullptr) == SYMPIX_EINVAL);
        CHECK(sympix_factor_diag(a, fake, nb - 1, nullptr, 0, fake, nu, ifake, da.ntiles, nullptr) == SYMPIX_ESIZE);
        CHECK(sympix_factor_diag(a, fake, nb, nullptr, nb, fake, nu, ifake, da.ntiles, nullptr) == SYMPIX_ESIZE);
        CHECK(sympix_factor_diag(a, fake, nb, fake, nb, fake, nu, ifake, da.ntiles + 1, nullptr) == SYMPIX_ESIZE);
        CHECK(sympix_factor_diag(a, nullptr, nb, nullptr, 0, fake, nu, ifake, da.ntiles, nullptr) == SYMPIX_EINVAL);
        CHECK(sympix_factor_diag(b, fake, 0, nullptr, 0, fake, 0, ifake, 0, nullptr) == SYMPIX_EUNSUPPORTED);
        CHECK(sympix_solve_diag(nullptr, fake, nu, fake, da.npix, fake, da.npix, nullptr) == SYMPIX_EINVAL);
        CHECK(sympix_solve_diag(a, fake, nu, fake, da.npix - 1, fake, da.npix, nullptr) == SYMPIX_ESIZE);
        CHECK(sympix_solve_diag(a, fake, nu, fake, da.npix, fake + 8, da.npix, nullptr) == SYMPIX_EINVAL);
        CHECK(sympix_solve_diag(b, fake, 0, fake, 0, fake, 0, nullptr) == SYMPIX_EUNSUPPORTED);
    }
    sympix_sht_destroy(nullptr);
    sympix_grid_destroy(a);
    sympix_grid_destroy(b);
    sympix_grid_destroy(nullptr);
    sympix_cross_destroy(nullptr);
    sympix_kernel_destroy(nullptr);
    sympix_batch_destroy(nullptr);
    if (failures) {
        std::fprintf(stderr, "abi_host_check: %d failed checks\n", failures);
        return 1;
    }
    std::printf("abi_host_check OK\n");
    return 0;
}
