// C ABI of the SymPix library: argument checks, handle lifetimes, device
// tables and launches.  Declarations and contracts are in include/sympix.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../include/sympix.h"
#include "device.hpp"
#include "geometry.hpp"
#include "precond.hpp"
#include "sht.hpp"

using sympix::Geometry;
using sympix::UInfo;

namespace {

thread_local std::string g_last_error;

constexpr double kPi = 3.14159265358979323846;

sympix_status fail(sympix_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

sympix_status hip_fail(hipError_t e, const char *what) {
    return fail(SYMPIX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool sync_mode() {
    const char *v = std::getenv("SYMPIX_SYNC");
    return v && v[0] == '1';
}

// Allocation-failure injection for tests of the error paths: with the
// environment variable SYMPIX_FAIL_ALLOC=n, the n-th host allocation point
// reached since the variable took its current value (counting from 1) fails
// as an allocation would: the call returns ENOMEM and creates no handle.
// Allocation points: every handle the library allocates and every table build
// (grid, two-hop pattern, two-grid pair, kernel, batch).
bool injected_alloc_failure() {
    static std::mutex mu;
    static std::string last;
    static long count = 0;
    const char *v = std::getenv("SYMPIX_FAIL_ALLOC");
    std::lock_guard<std::mutex> lock(mu);
    if (!v || !*v) {
        last.clear();
        count = 0;
        return false;
    }
    if (last != v) {
        last = v;
        count = 0;
    }
    return ++count == std::strtol(v, nullptr, 10);
}

// Device copies of the grid tables, one set per device that used the grid.
struct DevGrid {
    double *ring_theta = nullptr;
    double *ring_sin = nullptr;
    UInfo *uinfo = nullptr;
    int32_t *blk_uid = nullptr;
    int32_t *exp_blk = nullptr;
    int32_t *exp_items = nullptr;
    sympix::DevClass *classes = nullptr;
    int32_t *class_terms = nullptr;
    int32_t *class_blk = nullptr;
    int32_t *class_itab = nullptr;
    int32_t *mtiles = nullptr;          // member tiles, class order (batch work items)
    int32_t *mtiles32 = nullptr;
    int32_t *gtiles = nullptr;          // the same as the class-grid launch's dispatch tables
    int32_t *gtiles32 = nullptr;
    int32_t *conv_chunks = nullptr;
    int32_t *conv_slots = nullptr;
    int32_t *diag_blk = nullptr;        // per tile: its stored block (J, J)
};

template <class T>
hipError_t upload(T **dst, const T *src, size_t n) {
    *dst = nullptr;
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, n * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

void free_dev(DevGrid &d) {
    hipFree(d.ring_theta);
    hipFree(d.ring_sin);
    hipFree(d.uinfo);
    hipFree(d.blk_uid);
    hipFree(d.exp_blk);
    hipFree(d.exp_items);
    hipFree(d.classes);
    hipFree(d.class_terms);
    hipFree(d.class_blk);
    hipFree(d.class_itab);
    hipFree(d.mtiles);
    hipFree(d.mtiles32);
    hipFree(d.gtiles);
    hipFree(d.gtiles32);
    hipFree(d.conv_chunks);
    hipFree(d.conv_slots);
    hipFree(d.diag_blk);
    d = DevGrid();
}

// Device copies of the class tables of a further stored-block pattern.
struct DevClasses {
    sympix::DevClass *classes = nullptr;
    int32_t *class_terms = nullptr;
    int32_t *class_blk = nullptr;
    int32_t *class_itab = nullptr;
    int32_t *gtiles = nullptr;          // dispatch table of the class-grid launch
};

void free_dev_classes(DevClasses &d) {
    hipFree(d.classes);
    hipFree(d.class_terms);
    hipFree(d.class_blk);
    hipFree(d.class_itab);
    hipFree(d.gtiles);
    d = DevClasses();
}

}  // namespace

struct sympix_grid {
    Geometry geo;
    mutable std::mutex mu;
    mutable std::map<int, DevGrid> dev;
    mutable std::unique_ptr<sympix::Pattern> two_hop;    // built on first use
    mutable std::map<int, DevClasses> dev_two_hop;
};

struct sympix_cross;

struct sympix_kernel {
    const sympix_grid *g = nullptr;       // owner: one grid, or
    const sympix_cross *x = nullptr;      // a pair of grids (B-hat = Y_2 B Y_1^T)
    int device = 0;
    int32_t n_nodes = 0;
    double h = 0.0, inv_h = 0.0, y_cut = 0.0;
    double *coef = nullptr;
    double *table = nullptr;
    double *u64 = nullptr;
    float *ut32 = nullptr;
    double *u64t = nullptr;
    void *block = nullptr;    // one stream-ordered allocation holding all of the above
};

namespace {

// Upload the grid's tables to the current device once (blocking copies, so
// every stream sees them afterwards).  With create = false only an existing
// upload is returned (EINVAL if there is none): nothing is allocated.
sympix_status device_tables(const sympix_grid *g, int device, const DevGrid **out, bool create = true) {
    std::lock_guard<std::mutex> lock(g->mu);
    auto it = g->dev.find(device);
    if (it != g->dev.end()) {
        *out = &it->second;
        return SYMPIX_OK;
    }
    if (!create) return fail(SYMPIX_EINVAL, "the grid's tables are not on this device (tabulate a kernel first)");
    const Geometry &geo = g->geo;
    std::vector<UInfo> uinfo(geo.nunique());
    for (int64_t u = 0; u < geo.nunique(); ++u) {
        const int64_t I = geo.rep_i[u], J = geo.rep_j[u];
        const int bI = geo.tile_band[I], bJ = geo.tile_band[J];
        UInfo x;
        x.ring0_i = geo.band_ring0[bI];
        x.ring0_j = geo.band_ring0[bJ];
        x.n_i = geo.k * geo.band_tiles[bI];
        x.n_j = geo.k * geo.band_tiles[bJ];
        x.p0_i = (int32_t)((I - geo.band_tile0[bI]) * geo.k);
        x.p0_j = (int32_t)((J - geo.band_tile0[bJ]) * geo.k);
        x.pad0 = x.pad1 = 0;
        uinfo[u] = x;
    }
    static_assert(sizeof(sympix::DevClass) == sizeof(sympix::BlockClass), "class layout");
    DevGrid d;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(&d.ring_theta, geo.theta.data(), geo.theta.size());
    if (e == hipSuccess) e = upload(&d.ring_sin, geo.sin_theta.data(), geo.sin_theta.size());
    if (e == hipSuccess) e = upload(&d.uinfo, uinfo.data(), uinfo.size());
    if (e == hipSuccess) e = upload(&d.blk_uid, geo.blk_uid.data(), geo.blk_uid.size());
    if (e == hipSuccess) e = upload(&d.exp_blk, geo.exp_blk.data(), geo.exp_blk.size());
    if (e == hipSuccess) e = upload(&d.exp_items, geo.exp_items.data(), geo.exp_items.size());
    if (e == hipSuccess)
        e = upload(&d.classes, reinterpret_cast<const sympix::DevClass *>(geo.cls.classes.data()),
                   geo.cls.classes.size());
    if (e == hipSuccess) e = upload(&d.class_terms, geo.cls.class_terms.data(), geo.cls.class_terms.size());
    if (e == hipSuccess) e = upload(&d.class_blk, geo.cls.class_blk.data(), geo.cls.class_blk.size());
    if (e == hipSuccess) e = upload(&d.class_itab, geo.cls.class_itab.data(), geo.cls.class_itab.size());
    if (e == hipSuccess) e = upload(&d.mtiles, geo.cls.mtiles.data(), geo.cls.mtiles.size());
    if (e == hipSuccess) e = upload(&d.mtiles32, geo.cls.mtiles32.data(), geo.cls.mtiles32.size());
    if (e == hipSuccess) e = upload(&d.gtiles, geo.cls.gtiles.data(), geo.cls.gtiles.size());
    if (e == hipSuccess) e = upload(&d.gtiles32, geo.cls.gtiles32.data(), geo.cls.gtiles32.size());
    if (e == hipSuccess) e = upload(&d.conv_chunks, geo.conv_chunks.data(), geo.conv_chunks.size());
    if (e == hipSuccess) e = upload(&d.conv_slots, geo.conv_slots.data(), geo.conv_slots.size());
    std::vector<int32_t> diag(geo.ntiles);
    for (int64_t J = 0; J < geo.ntiles; ++J) diag[J] = (int32_t)geo.blk_ptr[J];   // K ascending from K = J
    if (e == hipSuccess) e = upload(&d.diag_blk, diag.data(), diag.size());
    if (e != hipSuccess) {
        free_dev(d);
        return e == hipErrorOutOfMemory ? fail(SYMPIX_ENOMEM, "device allocation for grid tables failed")
                                        : hip_fail(e, "uploading grid tables");
    }
    auto res = g->dev.emplace(device, d);
    *out = &res.first->second;
    return SYMPIX_OK;
}

// The two-hop pattern of grid g (host tables built on first use) and, with
// device >= 0, its class tables on that device.
sympix_status two_hop_tables(const sympix_grid *g, int device, const sympix::Pattern **pat,
                             const DevClasses **dc) {
    std::lock_guard<std::mutex> lock(g->mu);
    if (!g->two_hop) {
        if (injected_alloc_failure()) return fail(SYMPIX_ENOMEM, "host allocation failed building the two-hop pattern");
        auto p = std::make_unique<sympix::Pattern>();
        std::string err;
        const int st = sympix::build_two_hop(g->geo, *p, err);
        if (st != 0) return fail((sympix_status)st, err);
        g->two_hop = std::move(p);
    }
    *pat = g->two_hop.get();
    if (device < 0) return SYMPIX_OK;
    auto it = g->dev_two_hop.find(device);
    if (it != g->dev_two_hop.end()) {
        *dc = &it->second;
        return SYMPIX_OK;
    }
    const sympix::ClassTables &ct = g->two_hop->cls;
    DevClasses d;
    hipError_t e = upload(&d.classes, reinterpret_cast<const sympix::DevClass *>(ct.classes.data()), ct.classes.size());
    if (e == hipSuccess) e = upload(&d.class_terms, ct.class_terms.data(), ct.class_terms.size());
    if (e == hipSuccess) e = upload(&d.class_blk, ct.class_blk.data(), ct.class_blk.size());
    if (e == hipSuccess) e = upload(&d.class_itab, ct.class_itab.data(), ct.class_itab.size());
    if (e == hipSuccess) e = upload(&d.gtiles, ct.gtiles.data(), ct.gtiles.size());
    if (e != hipSuccess) {
        free_dev_classes(d);
        return e == hipErrorOutOfMemory ? fail(SYMPIX_ENOMEM, "device allocation for the two-hop tables failed")
                                        : hip_fail(e, "uploading the two-hop tables");
    }
    auto res = g->dev_two_hop.emplace(device, d);
    *dc = &res.first->second;
    return SYMPIX_OK;
}

sympix_status after_launch(hipError_t e, hipStream_t st, const char *what) {
    if (e != hipSuccess) return hip_fail(e, what);
    if (sync_mode()) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    return SYMPIX_OK;
}

sympix::KTable ktable(const sympix_kernel *kr) {
    sympix::KTable kt;
    kt.table = kr->table;
    kt.n_nodes = kr->n_nodes;
    kt.inv_h = kr->inv_h;
    kt.y_cut = kr->y_cut;
    return kt;
}

// Stream-ordered release on the null stream: it follows all work already
// queued on blocking streams and does not stall the host.
void free_kernel(sympix_kernel *kr) {
    if (kr->block) {
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (have && cur != kr->device) hipSetDevice(kr->device);
        hipFreeAsync(kr->block, nullptr);
        if (have && cur != kr->device) hipSetDevice(cur);
    }
    delete kr;
}

// Pinned staging slots for the coefficient upload, so that it is an
// asynchronous copy in stream order (a pageable copy would wait for the
// device).  A slot is reused only after its previous copy has completed.
struct CoefSlot {
    double *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
std::mutex g_coef_mu;
std::map<int, std::vector<CoefSlot>> g_coef_slots;   // per device
std::map<int, size_t> g_coef_next;

hipError_t upload_coefficients(int device, const std::vector<double> &coef, double *dst, hipStream_t st) {
    std::lock_guard<std::mutex> lock(g_coef_mu);
    auto &ring = g_coef_slots[device];
    if (ring.empty()) ring.resize(8);
    CoefSlot &slot = ring[g_coef_next[device]++ % ring.size()];
    hipError_t e = hipSuccess;
    if (slot.pending) {
        e = hipEventSynchronize(slot.done);
        if (e != hipSuccess) return e;
        slot.pending = false;
    }
    if (!slot.done) {
        e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (slot.cap < coef.size()) {
        if (slot.host) hipHostFree(slot.host);
        slot.host = nullptr;
        slot.cap = 0;
        e = hipHostMalloc((void **)&slot.host, coef.size() * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        slot.cap = coef.size();
    }
    std::memcpy(slot.host, coef.data(), coef.size() * sizeof(double));
    e = hipMemcpyAsync(dst, slot.host, coef.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(slot.done, st);
    if (e == hipSuccess) slot.pending = true;
    return e;
}

sympix_status check_kernel_use(const sympix_grid *g, const sympix_kernel *kr) {
    if (!g || !kr) return fail(SYMPIX_EINVAL, "NULL grid or kernel");
    if (kr->g != g) return fail(SYMPIX_EINVAL, "kernel was tabulated for another grid");
    if (g->geo.k != 8) return fail(SYMPIX_EUNSUPPORTED, "device sampling is implemented for k = 8 only");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != kr->device) return fail(SYMPIX_EINVAL, "kernel lives on another device than the current one");
    return SYMPIX_OK;
}

// Launch a contraction whose tables are set in a (all but the N^-1 operand
// scratch): the scratch is the library's static array (noalloc) or a
// stream-ordered allocation of a.npix values in the operand format.
sympix_status launch_contraction(sympix::BtnbArgs &a, int device, int32_t prec, bool noalloc, hipStream_t st,
                                 const char *what) {
    a.wsplit[0] = a.wsplit[1] = a.wsplit[2] = nullptr;
    a.wf32 = nullptr;
    hipError_t e = hipSuccess;
    void *scratch = nullptr;
    bool owned = false;
    if (prec != SYMPIX_FP64) {
        if (noalloc) {
            // the static array: shared by every allocation-free call on this
            // device, fully rewritten (npix values per part) before it is read
            e = sympix::noalloc_scratch(device, &scratch);
            if (e != hipSuccess) return hip_fail(e, "address of the static N^-1 scratch");
        } else {
            // stream-ordered scratch for N^-1 in the MFMA operand format (FP32,
            // or three BF16 parts): concurrent calls stay independent
            const size_t bytes = (size_t)a.npix * (prec == SYMPIX_FP32 ? sizeof(float) : 3 * sizeof(uint16_t));
            e = hipMallocAsync(&scratch, bytes, st);
            if (e != hipSuccess)
                return e == hipErrorOutOfMemory ? fail(SYMPIX_ENOMEM, "device scratch for N^-1 operands")
                                                : hip_fail(e, "hipMallocAsync");
            owned = true;
        }
        if (prec == SYMPIX_FP32) {
            a.wf32 = (float *)scratch;
        } else {
            a.wsplit[0] = (uint16_t *)scratch;
            a.wsplit[1] = a.wsplit[0] + a.npix;
            a.wsplit[2] = a.wsplit[1] + a.npix;
        }
    }
    e = sympix::launch_btnb(prec, a, st);
    if (owned) {
        hipError_t ef = hipFreeAsync(scratch, st);
        if (e == hipSuccess) e = ef;
    }
    return after_launch(e, st, what);
}

// B-hat^T N^-1 B-hat into out_dev and, with a D-hat kernel d, the D-hat
// blocks into outD_dev, both written by one class-GEMM launch.  With noalloc
// the N^-1 operand scratch is the library's static device array and nothing
// is allocated (the grid's tables must already be on the device).
sympix_status sample_btnb(const sympix_grid *g, const sympix_kernel *d, const sympix_kernel *b,
                          const double *ninv_dev, int64_t ninv_len, int32_t prec, int32_t pattern,
                          double *outD_dev, int64_t outD_len, double *out_dev, int64_t out_len, void *stream,
                          const char *what, bool noalloc = false) {
    sympix_status s = check_kernel_use(g, b);
    if (s != SYMPIX_OK) return s;
    const Geometry &geo = g->geo;
    if (prec < SYMPIX_FP64 || prec > SYMPIX_BF16X6) return fail(SYMPIX_EINVAL, "unknown precision mode");
    if (pattern != SYMPIX_PATTERN_ONE_HOP && pattern != SYMPIX_PATTERN_TWO_HOP)
        return fail(SYMPIX_EINVAL, "unknown block pattern");
    if (ninv_len != geo.npix) return fail(SYMPIX_ESIZE, "ninv_len must be npix");
    if (noalloc && prec != SYMPIX_FP64 && geo.npix > sympix::kNoAllocMaxPix)
        return fail(SYMPIX_ESIZE, "the allocation-free call holds N^-1 operands for at most " +
                                      std::to_string(sympix::kNoAllocMaxPix) + " pixels (this grid has " +
                                      std::to_string(geo.npix) + "); use sympix_sample_BtNB");
    const sympix::Pattern *pat = nullptr;
    if (pattern == SYMPIX_PATTERN_TWO_HOP) {
        const DevClasses *unused = nullptr;
        s = two_hop_tables(g, -1, &pat, &unused);
        if (s != SYMPIX_OK) return s;
    }
    const int64_t nblocks = pat ? pat->nblocks() : geo.nblocks();
    const sympix::ClassTables &ct = pat ? pat->cls : geo.cls;
    const int64_t want = nblocks * sympix::kBlockElems;
    if (out_len != want || (d && outD_len != want)) return fail(SYMPIX_ESIZE, "output lengths must be nblocks * k^4");
    if ((geo.npix > 0 && !ninv_dev) || (out_len > 0 && !out_dev) || (d && out_len > 0 && !outD_dev))
        return fail(SYMPIX_EINVAL, "NULL device buffer");
    if (((uintptr_t)out_dev) % 16 || ((uintptr_t)ninv_dev) % 32 || ((uintptr_t)outD_dev) % 16)
        return fail(SYMPIX_EINVAL, "outputs must be 16-byte and ninv_dev 32-byte aligned");
    if (out_len > 0) {
        auto overlap = [](const void *p, size_t np, const void *q, size_t nq) {
            return (const char *)p < (const char *)q + nq && (const char *)q < (const char *)p + np;
        };
        const size_t ob = (size_t)out_len * sizeof(double), nb = (size_t)ninv_len * sizeof(double);
        if (overlap(out_dev, ob, ninv_dev, nb)) return fail(SYMPIX_EINVAL, "the output overlaps ninv_dev");
        if (d && (overlap(outD_dev, ob, out_dev, ob) || overlap(outD_dev, ob, ninv_dev, nb)))
            return fail(SYMPIX_EINVAL, "the D-hat output overlaps another buffer");
    }
    if (d && d->device != b->device) return fail(SYMPIX_EINVAL, "the two kernels live on different devices");
    const DevGrid *dg = nullptr;
    s = device_tables(g, b->device, &dg, !noalloc);
    if (s != SYMPIX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (ct.max_class_terms > sympix::kMaxClassTerms)
        return fail(SYMPIX_EUNSUPPORTED, "a block has more contraction tiles than the class GEMM supports");
    const bool fused = d != nullptr;
    sympix::BtnbArgs a;
    a.u64t = b->u64t;
    a.ut32 = b->ut32;
    if (pat) {
        const DevClasses *dc = nullptr;
        s = two_hop_tables(g, b->device, &pat, &dc);
        if (s != SYMPIX_OK) return s;
        a.classes = dc->classes;
        a.class_terms = dc->class_terms;
        a.class_blk = dc->class_blk;
        a.class_itab = dc->class_itab;
        a.mtiles = dc->gtiles;
    } else {
        a.classes = dg->classes;
        a.class_terms = dg->class_terms;
        a.class_blk = dg->class_blk;
        a.class_itab = dg->class_itab;
        a.mtiles = dg->gtiles;
    }
    a.nmtiles = (int64_t)ct.gtiles.size() / 4;
    // A short FP64 launch runs faster on tiles of at most 32 rows: twice the tiles to
    // balance over the CUs, and the FP64 kernel keeps its full speed on half tiles
    if (!pat && prec == SYMPIX_FP64 && (int64_t)ct.mtiles.size() / 4 < sympix::kShortLaunchTiles) {
        a.mtiles = dg->gtiles32;
        a.nmtiles = (int64_t)ct.gtiles32.size() / 4;
    }
    a.nblocks = nblocks;
    a.npix = geo.npix;
    a.ninv = ninv_dev;
    a.out = out_dev;
    a.du64 = fused ? d->u64 : nullptr;
    a.blk_uid = fused ? dg->blk_uid : nullptr;
    a.outD = fused ? outD_dev : nullptr;
    return launch_contraction(a, b->device, prec, noalloc, st, what);
}

// What a kernel tabulation needs from its owner (one grid or a pair): the band
// limit of the series, the largest y between paired pixels, and the unique
// blocks with their ring tables on the device.
struct TabSource {
    int32_t lmax;
    double y_pattern_max;
    int64_t nunique;
    const UInfo *uinfo;
    const double *ring_theta, *ring_sin;
};

sympix_status tabulate(const TabSource &src, const sympix_grid *g, const sympix_cross *x, int device,
                       const double *coef_l, int32_t ncoef, double radius, int32_t n_nodes, hipStream_t st,
                       sympix_kernel **out) {
    if (ncoef < 1) return fail(SYMPIX_ESIZE, "ncoef must be >= 1");
    if (n_nodes == 0) n_nodes = 65536;
    if (n_nodes < 64) return fail(SYMPIX_EINVAL, "n_nodes must be >= 64");
    if (!(radius == radius)) return fail(SYMPIX_EINVAL, "radius is NaN");
    for (int32_t l = 0; l < ncoef; ++l)
        if (!std::isfinite(coef_l[l])) return fail(SYMPIX_EINVAL, "coefficients must be finite");
    sympix_kernel *kr = injected_alloc_failure() ? nullptr : new (std::nothrow) sympix_kernel();
    if (!kr) return fail(SYMPIX_ENOMEM, "host allocation failed");
    kr->g = g;
    kr->x = x;
    kr->device = device;
    kr->n_nodes = n_nodes;
    double y_dom = src.y_pattern_max;
    kr->y_cut = INFINITY;
    if (radius > 0) {
        const double sr = std::sin(0.5 * radius);
        kr->y_cut = 2.0 * sr * sr;
        if (kr->y_cut < y_dom) y_dom = kr->y_cut;
    }
    // nodes uniform in s = sqrt(y) up to the domain end plus a little slack for
    // device rounding of y; the last interval keeps one spare node
    const double s_top = std::fmax(std::sqrt(y_dom) * (1.0 + 1e-6), 1e-300);
    kr->h = s_top / (double)(n_nodes - 5);
    kr->inv_h = 1.0 / kr->h;

    const int32_t lmax = src.lmax;
    std::vector<double> coef(lmax + 1, 0.0);
    for (int32_t l = 0; l <= lmax && l < ncoef; ++l) coef[l] = coef_l[l];
    const size_t nu = (size_t)src.nunique * sympix::kBlockElems;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_table = up(coef.size() * sizeof(double));
    const size_t o_u64 = o_table + up((size_t)n_nodes * sizeof(double));
    const size_t o_u64t = o_u64 + up(nu * sizeof(double));
    const size_t o_ut32 = o_u64t + up(nu * sizeof(double));
    const size_t total = o_ut32 + up(nu * sizeof(float));
    hipError_t e = hipMallocAsync(&kr->block, total, st);
    if (e != hipSuccess) {
        kr->block = nullptr;
        free_kernel(kr);
        return e == hipErrorOutOfMemory ? fail(SYMPIX_ENOMEM, "device allocation for the kernel failed")
                                        : hip_fail(e, "hipMallocAsync");
    }
    char *base = (char *)kr->block;
    kr->coef = (double *)base;
    kr->table = (double *)(base + o_table);
    kr->u64 = (double *)(base + o_u64);
    kr->u64t = (double *)(base + o_u64t);
    kr->ut32 = (float *)(base + o_ut32);
    e = upload_coefficients(device, coef, kr->coef, st);
    if (e != hipSuccess) {
        hipStreamSynchronize(st);
        free_kernel(kr);
        return hip_fail(e, "copying coefficients");
    }
    e = sympix::launch_tabulate(kr->coef, lmax, kr->h, kr->table, n_nodes, st);
    if (e == hipSuccess)
        e = sympix::launch_unique_eval(ktable(kr), src.uinfo, src.nunique, src.ring_theta, src.ring_sin, kr->u64,
                                       kr->u64t, kr->ut32, st);
    sympix_status s = after_launch(e, st, "tabulate / unique-block evaluation");
    if (s != SYMPIX_OK) {
        hipStreamSynchronize(st);
        free_kernel(kr);
        return s;
    }
    *out = kr;
    return SYMPIX_OK;
}

}  // namespace

extern "C" {

const char *sympix_last_error(void) { return g_last_error.c_str(); }

sympix_status sympix_grid_create(int32_t lmax, int32_t k, double polar_margin, sympix_grid **out) {
    if (!out) return fail(SYMPIX_EINVAL, "out is NULL");
    *out = nullptr;
    sympix_grid *g = injected_alloc_failure() ? nullptr : new (std::nothrow) sympix_grid();
    if (!g) return fail(SYMPIX_ENOMEM, "host allocation failed");
    std::string err;
    int rc = injected_alloc_failure() ? (err = "host allocation failed while building the grid (injected)", -3)
                                      : sympix::build_geometry(lmax, k, polar_margin, g->geo, err);
    if (rc != 0) {
        delete g;
        return fail((sympix_status)rc, err);
    }
    *out = g;
    g_last_error.clear();
    return SYMPIX_OK;
}

void sympix_grid_destroy(sympix_grid *g) {
    if (!g) return;
    for (auto &kv : g->dev) free_dev(kv.second);
    for (auto &kv : g->dev_two_hop) free_dev_classes(kv.second);
    delete g;
}

sympix_status sympix_grid_dims(const sympix_grid *g, sympix_dims *out) {
    if (!g || !out) return fail(SYMPIX_EINVAL, "NULL argument");
    const Geometry &s = g->geo;
    out->lmax = s.lmax;
    out->k = s.k;
    out->nrings = s.nrings;
    out->nbands_hemi = s.nbands_hemi;
    out->npix = s.npix;
    out->ntiles = s.ntiles;
    out->nadjacency = (int64_t)s.adj_col.size();
    out->nblocks = s.nblocks();
    out->nterms = (int64_t)s.terms.size();
    out->nunique = s.nunique();
    out->polar_margin = s.margin;
    out->y_pattern_max = s.y_pattern_max;
    return SYMPIX_OK;
}

sympix_status sympix_grid_rings(const sympix_grid *g, double *theta, double *weight,
                                int32_t *npix_ring, int64_t *first_pix) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &s = g->geo;
    const size_t n = (size_t)s.nrings;
    if (theta) std::memcpy(theta, s.theta.data(), n * sizeof(double));
    if (weight) std::memcpy(weight, s.weight.data(), n * sizeof(double));
    if (npix_ring) std::memcpy(npix_ring, s.ring_npix.data(), n * sizeof(int32_t));
    if (first_pix) std::memcpy(first_pix, s.ring_first_pix.data(), n * sizeof(int64_t));
    return SYMPIX_OK;
}

sympix_status sympix_grid_bands(const sympix_grid *g, int32_t *tiles, int32_t *alpha,
                                int32_t *first_ring) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &s = g->geo;
    const size_t n = s.band_tiles.size();
    if (tiles) std::memcpy(tiles, s.band_tiles.data(), n * sizeof(int32_t));
    if (alpha) std::memcpy(alpha, s.band_alpha.data(), n * sizeof(int32_t));
    if (first_ring) std::memcpy(first_ring, s.band_ring0.data(), n * sizeof(int32_t));
    return SYMPIX_OK;
}

sympix_status sympix_grid_pixels(const sympix_grid *g, double *theta, double *phi) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &s = g->geo;
    const int64_t k = s.k;
    for (size_t b = 0; b < s.band_tiles.size(); ++b) {
        const int64_t n = k * s.band_tiles[b];          // pixels on each ring of the band
        const int64_t pix0 = s.band_tile0[b] * k * k;
        for (int64_t r = 0; r < k; ++r) {
            const double th = s.theta[s.band_ring0[b] + r];
            for (int64_t p = 0; p < n; ++p) {
                const int64_t idx = pix0 + (p / k) * k * k + (p % k) * k + r;   // tile, column, ring
                if (theta) theta[idx] = th;
                if (phi) phi[idx] = 2.0 * kPi * ((double)p + 0.5) / (double)n;
            }
        }
    }
    return SYMPIX_OK;
}

sympix_status sympix_grid_neighbours(const sympix_grid *g, int64_t *row_ptr, int32_t *col) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &s = g->geo;
    if (row_ptr) std::memcpy(row_ptr, s.adj_ptr.data(), s.adj_ptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, s.adj_col.data(), s.adj_col.size() * sizeof(int32_t));
    return SYMPIX_OK;
}

sympix_status sympix_grid_blocks(const sympix_grid *g, int64_t *row_ptr, int32_t *col) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &s = g->geo;
    if (row_ptr) std::memcpy(row_ptr, s.blk_ptr.data(), s.blk_ptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, s.blk_col.data(), s.blk_col.size() * sizeof(int32_t));
    return SYMPIX_OK;
}

sympix_status sympix_grid_pattern_blocks(const sympix_grid *g, int32_t pattern, int64_t *nblocks, int64_t *nterms,
                                        int64_t *row_ptr, int32_t *col) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const std::vector<int64_t> *ptr = &g->geo.blk_ptr;
    const std::vector<int32_t> *cols = &g->geo.blk_col;
    int64_t nt = (int64_t)g->geo.terms.size();
    if (pattern == SYMPIX_PATTERN_TWO_HOP) {
        const sympix::Pattern *pat = nullptr;
        const DevClasses *unused = nullptr;
        sympix_status s = two_hop_tables(g, -1, &pat, &unused);
        if (s != SYMPIX_OK) return s;
        ptr = &pat->blk_ptr;
        cols = &pat->blk_col;
        nt = (int64_t)pat->terms.size();
    } else if (pattern != SYMPIX_PATTERN_ONE_HOP) {
        return fail(SYMPIX_EINVAL, "unknown block pattern");
    }
    if (nblocks) *nblocks = (int64_t)cols->size();
    if (nterms) *nterms = nt;
    if (row_ptr) std::memcpy(row_ptr, ptr->data(), ptr->size() * sizeof(int64_t));
    if (col) std::memcpy(col, cols->data(), cols->size() * sizeof(int32_t));
    return SYMPIX_OK;
}

sympix_status sympix_grid_unique(const sympix_grid *g, int32_t *uid, int32_t *key_band_i,
                                 int32_t *key_band_j, int64_t *key_delta) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &s = g->geo;
    if (uid) std::memcpy(uid, s.adj_uid.data(), s.adj_uid.size() * sizeof(int32_t));
    if (key_band_i) std::memcpy(key_band_i, s.key_band_i.data(), s.key_band_i.size() * sizeof(int32_t));
    if (key_band_j) std::memcpy(key_band_j, s.key_band_j.data(), s.key_band_j.size() * sizeof(int32_t));
    if (key_delta) std::memcpy(key_delta, s.key_delta.data(), s.key_delta.size() * sizeof(int64_t));
    return SYMPIX_OK;
}

sympix_status sympix_kernel_tabulate(const sympix_grid *g, const double *coef_l, int32_t ncoef,
                                     double radius, int32_t n_nodes, void *stream,
                                     sympix_kernel **out) {
    if (!out) return fail(SYMPIX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || !coef_l) return fail(SYMPIX_EINVAL, "NULL grid or coefficients");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const DevGrid *dg = nullptr;
    sympix_status s = device_tables(g, device, &dg);
    if (s != SYMPIX_OK) return s;
    const Geometry &geo = g->geo;
    TabSource src{geo.lmax, geo.y_pattern_max, geo.nunique(), dg->uinfo, dg->ring_theta, dg->ring_sin};
    return tabulate(src, g, nullptr, device, coef_l, ncoef, radius, n_nodes, (hipStream_t)stream, out);
}

void sympix_kernel_destroy(sympix_kernel *kr) {
    if (kr) free_kernel(kr);
}

sympix_status sympix_kernel_eval(const sympix_kernel *kr, const double *y_dev, double *out_dev,
                                 int64_t n, void *stream) {
    if (!kr || (n > 0 && (!y_dev || !out_dev))) return fail(SYMPIX_EINVAL, "NULL argument");
    if (n < 0) return fail(SYMPIX_ESIZE, "n < 0");
    hipStream_t st = (hipStream_t)stream;
    return after_launch(sympix::launch_eval(ktable(kr), y_dev, out_dev, n, st), st, "kernel_eval");
}

sympix_status sympix_sample_D(const sympix_grid *g, const sympix_kernel *d, double *out_dev,
                              int64_t out_len, void *stream) {
    sympix_status s = check_kernel_use(g, d);
    if (s != SYMPIX_OK) return s;
    const Geometry &geo = g->geo;
    if (out_len != geo.nblocks() * sympix::kBlockElems)
        return fail(SYMPIX_ESIZE, "out_len must be nblocks * k^4");
    if (out_len > 0 && !out_dev) return fail(SYMPIX_EINVAL, "out_dev is NULL");
    if (((uintptr_t)out_dev) % 16) return fail(SYMPIX_EINVAL, "out_dev must be 16-byte aligned");
    const DevGrid *dg = nullptr;
    s = device_tables(g, d->device, &dg);
    if (s != SYMPIX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return after_launch(sympix::launch_expand(d->u64, dg->exp_items, (int64_t)geo.exp_items.size() / 4, dg->exp_blk, out_dev, st), st,
                        "sample_D");
}

sympix_status sympix_factor_diag(const sympix_grid *g, const double *D_dev, int64_t D_len, const double *C_dev,
                                 int64_t C_len, double *U_dev, int64_t U_len, int32_t *info_dev, int64_t info_len,
                                 void *stream) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &geo = g->geo;
    if (geo.k != 8) return fail(SYMPIX_EUNSUPPORTED, "device kernels are built for k = 8");
    const int64_t nb = geo.nblocks() * sympix::kBlockElems, nu = geo.ntiles * sympix::kBlockElems;
    if (D_len != nb || (C_dev ? C_len != nb : C_len != 0) || U_len != nu || info_len != geo.ntiles)
        return fail(SYMPIX_ESIZE, "D_len and C_len must be nblocks * k^4 (C_len 0 without C), U_len ntiles * k^4, "
                                  "info_len ntiles");
    if (geo.ntiles > 0 && (!D_dev || !U_dev || !info_dev)) return fail(SYMPIX_EINVAL, "NULL device buffer");
    if (((uintptr_t)D_dev) % 16 || ((uintptr_t)C_dev) % 16 || ((uintptr_t)U_dev) % 16 || ((uintptr_t)info_dev) % 4)
        return fail(SYMPIX_EINVAL, "misaligned device buffer");
    auto overlaps = [](const void *a, int64_t na, const void *b, int64_t nb2) {
        return a && b && (const char *)a < (const char *)b + nb2 && (const char *)b < (const char *)a + na;
    };
    const int64_t bU = U_len * 8, bI = info_len * 4;
    if (overlaps(U_dev, bU, D_dev, D_len * 8) || overlaps(U_dev, bU, C_dev, C_len * 8) ||
        overlaps(info_dev, bI, D_dev, D_len * 8) || overlaps(info_dev, bI, C_dev, C_len * 8) ||
        overlaps(info_dev, bI, U_dev, bU))
        return fail(SYMPIX_EINVAL, "an output overlaps another buffer");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const DevGrid *dg = nullptr;
    sympix_status s = device_tables(g, device, &dg);
    if (s != SYMPIX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return after_launch(sympix::launch_factor_diag(D_dev, C_dev, dg->diag_blk, geo.ntiles, U_dev, info_dev, st), st,
                        "factor_diag");
}

sympix_status sympix_solve_diag(const sympix_grid *g, const double *U_dev, int64_t U_len, const double *r_dev,
                                int64_t r_len, double *x_dev, int64_t x_len, void *stream) {
    if (!g) return fail(SYMPIX_EINVAL, "NULL grid");
    const Geometry &geo = g->geo;
    if (geo.k != 8) return fail(SYMPIX_EUNSUPPORTED, "device kernels are built for k = 8");
    if (U_len != geo.ntiles * sympix::kBlockElems || r_len != geo.npix || x_len != geo.npix)
        return fail(SYMPIX_ESIZE, "U_len must be ntiles * k^4, r_len and x_len npix");
    if (geo.ntiles > 0 && (!U_dev || !r_dev || !x_dev)) return fail(SYMPIX_EINVAL, "NULL device buffer");
    if (((uintptr_t)U_dev) % 16 || ((uintptr_t)r_dev) % 16 || ((uintptr_t)x_dev) % 16)
        return fail(SYMPIX_EINVAL, "misaligned device buffer");
    if (x_dev != r_dev && x_dev && r_dev && r_dev < x_dev + x_len && x_dev < r_dev + r_len)
        return fail(SYMPIX_EINVAL, "x_dev overlaps r_dev without being it");
    if (x_dev && U_dev && (const double *)x_dev < U_dev + U_len && U_dev < (const double *)x_dev + x_len)
        return fail(SYMPIX_EINVAL, "x_dev overlaps U_dev");
    hipStream_t st = (hipStream_t)stream;
    return after_launch(sympix::launch_solve_diag(U_dev, r_dev, x_dev, geo.ntiles, st), st, "solve_diag");
}

sympix_status sympix_convolve(const sympix_grid *g, const sympix_kernel *b, const double *f_dev,
                              int64_t f_len, double *out_dev, int64_t out_len, void *stream) {
    sympix_status s = check_kernel_use(g, b);
    if (s != SYMPIX_OK) return s;
    const Geometry &geo = g->geo;
    if (f_len != geo.npix || out_len != geo.npix) return fail(SYMPIX_ESIZE, "f_len and out_len must be npix");
    if (geo.npix > 0 && (!f_dev || !out_dev)) return fail(SYMPIX_EINVAL, "NULL device buffer");
    if (((uintptr_t)f_dev) % 16 || ((uintptr_t)out_dev) % 16)
        return fail(SYMPIX_EINVAL, "f_dev and out_dev must be 16-byte aligned");
    if (f_dev && out_dev && f_dev < out_dev + out_len && out_dev < f_dev + f_len)
        return fail(SYMPIX_EINVAL, "f_dev and out_dev overlap");
    const DevGrid *dg = nullptr;
    s = device_tables(g, b->device, &dg);
    if (s != SYMPIX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return after_launch(sympix::launch_convolve(b->u64, dg->conv_chunks, (int64_t)geo.conv_chunks.size() / 4,
                                                dg->conv_slots, f_dev, out_dev, st),
                        st, "convolve");
}

sympix_status sympix_sample_BtNB(const sympix_grid *g, const sympix_kernel *b, const double *ninv_dev,
                                 int64_t ninv_len, int32_t prec, double *out_dev, int64_t out_len,
                                 void *stream) {
    return sample_btnb(g, nullptr, b, ninv_dev, ninv_len, prec, SYMPIX_PATTERN_ONE_HOP, nullptr, 0, out_dev, out_len,
                       stream, "sample_BtNB");
}

sympix_status sympix_sample_BtNB_noalloc(const sympix_grid *g, const sympix_kernel *b, const double *ninv_dev,
                                         int64_t ninv_len, int32_t prec, double *out_dev, int64_t out_len,
                                         void *stream) {
    return sample_btnb(g, nullptr, b, ninv_dev, ninv_len, prec, SYMPIX_PATTERN_ONE_HOP, nullptr, 0, out_dev, out_len,
                       stream, "sample_BtNB_noalloc", true);
}

sympix_status sympix_sample_BtNB_pattern(const sympix_grid *g, const sympix_kernel *b, const double *ninv_dev,
                                         int64_t ninv_len, int32_t prec, int32_t pattern, double *out_dev,
                                         int64_t out_len, void *stream) {
    return sample_btnb(g, nullptr, b, ninv_dev, ninv_len, prec, pattern, nullptr, 0, out_dev, out_len, stream,
                       "sample_BtNB_pattern");
}

sympix_status sympix_sample_D_BtNB(const sympix_grid *g, const sympix_kernel *d, const sympix_kernel *b,
                                   const double *ninv_dev, int64_t ninv_len, int32_t prec, double *outD_dev,
                                   int64_t outD_len, double *outC_dev, int64_t outC_len, void *stream) {
    sympix_status s = check_kernel_use(g, d);
    if (s != SYMPIX_OK) return s;
    return sample_btnb(g, d, b, ninv_dev, ninv_len, prec, SYMPIX_PATTERN_ONE_HOP, outD_dev, outD_len, outC_dev,
                       outC_len, stream, "sample_D_BtNB");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches (a10): many problems, one captured graph.
// ---------------------------------------------------------------------------
struct sympix_batch {
    int device = 0;
    int32_t nprob = 0;
    int32_t prec = SYMPIX_FP32;
    int32_t schedule = SYMPIX_SCHED_XCD_QUEUES;
    int32_t tiling = SYMPIX_TILES_64;
    int32_t nworkgroups = 0;
    // per tile shape (sympix_tiling): problem descriptors, dispatch tables,
    // work items in natural order
    std::vector<sympix::ProblemDesc64> hdesc64[SYMPIX_NTILINGS]; // FP64
    std::vector<sympix::ProblemDesc> hdesc[SYMPIX_NTILINGS];     // FP32
    std::vector<sympix::ProblemDescB> hdescb[SYMPIX_NTILINGS];   // split BF16
    std::vector<const int32_t *> gtiles[SYMPIX_NTILINGS];   // per problem: the class-grid dispatch table
    std::vector<int64_t> ngtiles[SYMPIX_NTILINGS];
    std::vector<int32_t> item_prob[SYMPIX_NTILINGS], item_tile[SYMPIX_NTILINGS], item_cost[SYMPIX_NTILINGS];
    std::vector<uint16_t *> wsplit;                // split BF16: 3 N^-1 parts per problem
    std::vector<const double *> ninv;
    std::vector<int64_t> npix;
    sympix::ProblemDesc64 *d_desc64[SYMPIX_NTILINGS] = {};
    sympix::ProblemDesc *d_desc[SYMPIX_NTILINGS] = {};
    int32_t *d_items = nullptr;
    int32_t *d_qb = nullptr;
    int32_t *d_counters = nullptr;
    float *d_wf = nullptr;
    sympix::ProblemDescB *d_descb[SYMPIX_NTILINGS] = {};
    uint16_t *d_wsplit = nullptr;
    hipStream_t cap = nullptr;
    hipEvent_t done = nullptr;          // recorded after every launch of the graph
    bool launched = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string shape;
};

namespace {

constexpr int kBatchQueues = 8;   // one per XCD

std::mutex g_tune_mu;
std::map<std::string, int32_t> g_tune_cache;   // batch shape -> plan (schedule + NSCHED tiling)

// On-disk tuner cache: with SYMPIX_TUNE_CACHE=<file>, plans chosen by
// sympix_batch_tune are kept in that text file, one "<key>\t<plan>" line per
// batch shape (key: the gfx architecture, the HIP runtime version, the mode
// and every problem's lmax and block count), and sympix_batch_create starts
// from a plan found there.  The file is rewritten whole on every update
// (write to a temporary file, then rename); concurrent writers: last one wins.
std::string tune_cache_file() {
    const char *v = std::getenv("SYMPIX_TUNE_CACHE");
    return v ? std::string(v) : std::string();
}

std::map<std::string, int32_t> read_tune_file(const std::string &path) {
    std::map<std::string, int32_t> out;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        const size_t tab = l.rfind('\t');
        if (tab == std::string::npos || tab == 0) continue;
        char *end = nullptr;
        const long plan = std::strtol(l.c_str() + tab + 1, &end, 10);
        if (end == l.c_str() + tab + 1 || *end != '\0') continue;
        if (plan < 0 || plan >= SYMPIX_NSCHED * SYMPIX_NTILINGS) continue;
        out[l.substr(0, tab)] = (int32_t)plan;
    }
    std::fclose(f);
    return out;
}

bool write_tune_file(const std::string &path, const std::string &key, int32_t plan) {
    std::map<std::string, int32_t> all = read_tune_file(path);
    all[key] = plan;
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    bool ok = true;
    for (auto &kv : all) ok = ok && std::fprintf(f, "%s\t%d\n", kv.first.c_str(), kv.second) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (ok) ok = std::rename(tmp.c_str(), path.c_str()) == 0;
    if (!ok) std::remove(tmp.c_str());
    return ok;
}

void free_batch(sympix_batch *bt) {
    if (bt->exec) hipGraphExecDestroy(bt->exec);
    if (bt->graph) hipGraphDestroy(bt->graph);
    if (bt->cap) hipStreamDestroy(bt->cap);
    if (bt->done) hipEventDestroy(bt->done);
    for (int t = 0; t < SYMPIX_NTILINGS; ++t) {
        hipFree(bt->d_desc64[t]);
        hipFree(bt->d_desc[t]);
        hipFree(bt->d_descb[t]);
    }
    hipFree(bt->d_items);
    hipFree(bt->d_qb);
    hipFree(bt->d_counters);
    hipFree(bt->d_wf);
    hipFree(bt->d_wsplit);
    delete bt;
}

// Order the work items of tile shape t and bound the queues for schedule s,
// then capture the batch's launches into a fresh graph.
sympix_status capture_batch(sympix_batch *bt, int32_t s, int32_t t) {
    // the tables below are rewritten with blocking copies on the null stream,
    // which do not wait for a launch on a non-blocking stream: wait for the
    // batch's last launch first, whichever stream it was queued on
    if (bt->launched) {
        hipError_t ew = hipEventSynchronize(bt->done);
        if (ew != hipSuccess) return hip_fail(ew, "waiting for the batch's last launch");
        bt->launched = false;
    }
    const std::vector<int32_t> &item_prob = bt->item_prob[t], &item_tile = bt->item_tile[t],
                               &item_cost = bt->item_cost[t];
    const int64_t nitems = (int64_t)item_prob.size();
    std::vector<int64_t> order(nitems);
    std::iota(order.begin(), order.end(), 0);
    std::vector<int32_t> qb;
    if (s == SYMPIX_SCHED_XCD_QUEUES) {
        // contiguous ranges of equal work (sum of contraction tiles per item)
        const double total = std::accumulate(item_cost.begin(), item_cost.end(), 0.0);
        qb.push_back(0);
        double run = 0.0;
        int64_t i = 0;
        for (int q = 1; q < kBatchQueues; ++q) {
            while (i < nitems && run + 0.5 * item_cost[i] < total * q / kBatchQueues) run += item_cost[i++];
            qb.push_back((int32_t)i);
        }
        qb.push_back((int32_t)nitems);
    } else if (s == SYMPIX_SCHED_GLOBAL_LPT) {
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t a, int64_t b) { return item_cost[a] > item_cost[b]; });
        qb = {0, (int32_t)nitems};
    } else {
        qb = {0, 0};
    }
    std::vector<int32_t> items(2 * nitems);
    for (int64_t i = 0; i < nitems; ++i) {
        items[2 * i] = item_prob[order[i]];
        items[2 * i + 1] = item_tile[order[i]];
    }
    hipError_t e = hipSuccess;
    if (nitems > 0) e = hipMemcpy(bt->d_items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->d_qb, qb.data(), qb.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "uploading batch work items");

    if (bt->exec) hipGraphExecDestroy(bt->exec);
    if (bt->graph) hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;

    sympix::BatchLaunch bl;
    bl.nprob = bt->nprob;
    bl.prec = bt->prec;
    bl.host_desc64 = bt->hdesc64[t].data();
    bl.desc64 = bt->d_desc64[t];
    bl.host_desc = bt->hdesc[t].data();
    bl.host_descb = bt->hdescb[t].data();
    bl.wsplit = bt->wsplit.data();
    bl.descb = bt->d_descb[t];
    bl.ninv = bt->ninv.data();
    bl.npix = bt->npix.data();
    bl.gtiles = bt->gtiles[t].data();
    bl.ngtiles = bt->ngtiles[t].data();
    bl.desc = bt->d_desc[t];
    bl.items = bt->d_items;
    bl.nitems = nitems;
    bl.qb = bt->d_qb;
    bl.nq = (int32_t)qb.size() - 1;
    bl.counters = bt->d_counters;
    bl.persistent = s != SYMPIX_SCHED_PER_PROBLEM;
    bl.nworkgroups = bt->nworkgroups;

    e = hipStreamBeginCapture(bt->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t el = sympix::launch_batch(bl, bt->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(bt->cap, &graph);
    if (el != hipSuccess || e != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return hip_fail(el != hipSuccess ? el : e, "capturing the batch graph");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    bt->graph = graph;
    bt->exec = exec;
    bt->schedule = s;
    bt->tiling = t;
    return SYMPIX_OK;
}

}  // namespace

extern "C" {

sympix_status sympix_batch_create(const sympix_problem *p, int32_t n, int32_t prec, void *stream,
                                  sympix_batch **out) {
    if (!out) return fail(SYMPIX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p || n < 1) return fail(SYMPIX_EINVAL, "need at least one problem");
    if (prec < SYMPIX_FP64 || prec > SYMPIX_BF16X6) return fail(SYMPIX_EINVAL, "unknown precision mode");
    const size_t ninv_align = prec == SYMPIX_FP64 ? 32 : 8;   // FP64 loads N^-1 in 32-byte vectors
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    for (int32_t i = 0; i < n; ++i) {
        sympix_status s = check_kernel_use(p[i].g, p[i].b);
        if (s != SYMPIX_OK) return fail(s, "problem " + std::to_string(i) + ": " + g_last_error);
        const Geometry &geo = p[i].g->geo;
        if (p[i].ninv_len != geo.npix)
            return fail(SYMPIX_ESIZE, "problem " + std::to_string(i) + ": ninv_len must be npix");
        if (p[i].out_len != geo.nblocks() * sympix::kBlockElems)
            return fail(SYMPIX_ESIZE, "problem " + std::to_string(i) + ": out_len must be nblocks * k^4");
        if ((geo.npix > 0 && !p[i].ninv_dev) || (p[i].out_len > 0 && !p[i].out_dev))
            return fail(SYMPIX_EINVAL, "problem " + std::to_string(i) + ": NULL device buffer");
        if (((uintptr_t)p[i].out_dev) % 16 || ((uintptr_t)p[i].ninv_dev) % ninv_align)
            return fail(SYMPIX_EINVAL, "problem " + std::to_string(i) + ": out_dev must be 16-byte and ninv_dev " +
                                           std::to_string(ninv_align) + "-byte aligned");
        if (geo.cls.max_class_terms > sympix::kMaxClassTerms)
            return fail(SYMPIX_EUNSUPPORTED, "a block has more contraction tiles than the class GEMM supports");
        if (p[i].out_len > 0)
            spans.emplace_back((uintptr_t)p[i].out_dev, (uintptr_t)(p[i].out_dev + p[i].out_len));
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return fail(SYMPIX_EINVAL, "problem outputs overlap");

    sympix_batch *bt = injected_alloc_failure() ? nullptr : new (std::nothrow) sympix_batch();
    if (!bt) return fail(SYMPIX_ENOMEM, "host allocation");
    bt->device = p[0].b->device;
    bt->nprob = n;
    bt->prec = prec;
    const bool f64 = prec == SYMPIX_FP64;
    const bool bf16 = prec == SYMPIX_BF16X3 || prec == SYMPIX_BF16X6;
    hipError_t e = hipSuccess;
    int64_t wf_total = 0;
    std::string shape;
    {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, bt->device);
        if (e != hipSuccess) {
            free_batch(bt);
            return hip_fail(e, "hipGetDeviceProperties");
        }
        static const char *mode_name[] = {"|fp64", "|fp32", "|bf16x3", "|bf16x6"};
        int rt = 0;
        if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
        shape = std::string(prop.gcnArchName) + "|hip" + std::to_string(rt) + mode_name[prec];
        int occ = 0;
        e = sympix::batch_occupancy(prec, &occ);
        if (e != hipSuccess) {
            free_batch(bt);
            return hip_fail(e, "occupancy query");
        }
        bt->nworkgroups = std::max(1, occ) * prop.multiProcessorCount;
    }
    for (int32_t i = 0; i < n; ++i) {
        const Geometry &geo = p[i].g->geo;
        const DevGrid *dg = nullptr;
        sympix_status s = device_tables(p[i].g, bt->device, &dg);
        if (s != SYMPIX_OK) {
            free_batch(bt);
            return s;
        }
        for (int t = 0; t < SYMPIX_NTILINGS; ++t) {
            const int32_t *dtiles = t == SYMPIX_TILES_64 ? dg->mtiles : dg->mtiles32;
            const std::vector<int32_t> &tiles = t == SYMPIX_TILES_64 ? geo.cls.mtiles : geo.cls.mtiles32;
            sympix::ProblemDesc64 d64{dtiles, dg->classes, dg->class_terms, dg->class_blk, dg->class_itab,
                                      p[i].b->u64t, p[i].ninv_dev, p[i].out_dev, nullptr, nullptr, nullptr};
            bt->hdesc64[t].push_back(d64);
            sympix::ProblemDesc d{dtiles, dg->classes, dg->class_terms, dg->class_blk, dg->class_itab,
                                  p[i].b->ut32, nullptr, p[i].out_dev, nullptr, nullptr, nullptr};
            bt->hdesc[t].push_back(d);
            sympix::ProblemDescB db{dtiles, dg->classes, dg->class_terms, dg->class_blk, dg->class_itab,
                                    p[i].b->ut32, {nullptr, nullptr, nullptr}, p[i].out_dev, nullptr, nullptr, nullptr};
            bt->hdescb[t].push_back(db);
            const int64_t nmt = (int64_t)tiles.size() / 4;
            const std::vector<int32_t> &gt = t == SYMPIX_TILES_64 ? geo.cls.gtiles : geo.cls.gtiles32;
            bt->gtiles[t].push_back(t == SYMPIX_TILES_64 ? dg->gtiles : dg->gtiles32);
            bt->ngtiles[t].push_back((int64_t)gt.size() / 4);
            for (int64_t k = 0; k < nmt; ++k) {
                bt->item_prob[t].push_back(i);
                bt->item_tile[t].push_back((int32_t)k);
                bt->item_cost[t].push_back(geo.cls.classes[tiles[4 * k]].nterms * tiles[4 * k + 2]);
            }
        }
        bt->ninv.push_back(p[i].ninv_dev);
        bt->npix.push_back(geo.npix);
        wf_total += geo.npix;
        shape += "|" + std::to_string(geo.lmax) + ":" + std::to_string(geo.nblocks());
    }
    bt->shape = shape;
    const int64_t nitems = (int64_t)std::max(bt->item_prob[0].size(), bt->item_prob[1].size());
    if (nitems >= (int64_t)INT32_MAX / 2) {
        free_batch(bt);
        return fail(SYMPIX_ESIZE, "too many work items for one batch");
    }
    for (int t = 0; t < SYMPIX_NTILINGS && e == hipSuccess; ++t) {
        if (f64) e = hipMalloc((void **)&bt->d_desc64[t], n * sizeof(sympix::ProblemDesc64));
        else e = hipMalloc((void **)&bt->d_desc[t], n * sizeof(sympix::ProblemDesc));
        if (e == hipSuccess && bf16) e = hipMalloc((void **)&bt->d_descb[t], n * sizeof(sympix::ProblemDescB));
    }
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_items, std::max<int64_t>(1, 2 * nitems) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_qb, (kBatchQueues + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_counters, kBatchQueues * sizeof(int32_t));
    if (bf16) {
        if (e == hipSuccess)
            e = hipMalloc((void **)&bt->d_wsplit, std::max<int64_t>(1, 3 * wf_total) * sizeof(uint16_t));
    } else if (!f64 && e == hipSuccess) {
        e = hipMalloc((void **)&bt->d_wf, std::max<int64_t>(1, wf_total) * sizeof(float));
    }
    if (e != hipSuccess) {
        free_batch(bt);
        return e == hipErrorOutOfMemory ? fail(SYMPIX_ENOMEM, "device allocation for the batch")
                                        : hip_fail(e, "hipMalloc");
    }
    int64_t off = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3 && bf16; ++k) bt->wsplit.push_back(bt->d_wsplit + k * wf_total + off);
        for (int t = 0; t < SYMPIX_NTILINGS; ++t) {
            if (bf16)
                for (int k = 0; k < 3; ++k) bt->hdescb[t][i].w[k] = bt->wsplit[3 * i + k];
            else if (!f64)
                bt->hdesc[t][i].wf = bt->d_wf + off;
        }
        off += bt->npix[i];
    }
    for (int t = 0; t < SYMPIX_NTILINGS && e == hipSuccess; ++t) {
        if (f64)
            e = hipMemcpy(bt->d_desc64[t], bt->hdesc64[t].data(), n * sizeof(sympix::ProblemDesc64),
                          hipMemcpyHostToDevice);
        else
            e = hipMemcpy(bt->d_desc[t], bt->hdesc[t].data(), n * sizeof(sympix::ProblemDesc), hipMemcpyHostToDevice);
        if (e == hipSuccess && bf16)
            e = hipMemcpy(bt->d_descb[t], bt->hdescb[t].data(), n * sizeof(sympix::ProblemDescB),
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&bt->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_batch(bt);
        return hip_fail(e, "batch set-up");
    }
    int32_t plan = SYMPIX_SCHED_XCD_QUEUES + SYMPIX_NSCHED * SYMPIX_TILES_64;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(bt->shape);
        if (it != g_tune_cache.end()) {
            plan = it->second;
        } else {
            const std::string path = tune_cache_file();
            if (!path.empty()) {
                const std::map<std::string, int32_t> disk = read_tune_file(path);
                auto d = disk.find(bt->shape);
                if (d != disk.end()) {
                    plan = d->second;
                    g_tune_cache[bt->shape] = plan;
                }
            }
        }
    }
    sympix_status s = capture_batch(bt, plan % SYMPIX_NSCHED, plan / SYMPIX_NSCHED);
    if (s != SYMPIX_OK) {
        free_batch(bt);
        return s;
    }
    *out = bt;
    return SYMPIX_OK;
}

sympix_status sympix_batch_set_schedule(sympix_batch *bt, int32_t s) {
    if (!bt) return fail(SYMPIX_EINVAL, "NULL batch");
    if (s < 0 || s >= SYMPIX_NSCHED) return fail(SYMPIX_EINVAL, "unknown schedule");
    return capture_batch(bt, s, bt->tiling);
}

sympix_status sympix_batch_set_tiling(sympix_batch *bt, int32_t t) {
    if (!bt) return fail(SYMPIX_EINVAL, "NULL batch");
    if (t < 0 || t >= SYMPIX_NTILINGS) return fail(SYMPIX_EINVAL, "unknown tiling");
    return capture_batch(bt, bt->schedule, t);
}

sympix_status sympix_batch_launch(sympix_batch *bt, void *stream) {
    if (!bt || !bt->exec) return fail(SYMPIX_EINVAL, "NULL batch");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != bt->device) return fail(SYMPIX_EINVAL, "batch lives on another device than the current one");
    hipStream_t st = (hipStream_t)stream;
    e = hipGraphLaunch(bt->exec, st);
    if (e == hipSuccess) e = hipEventRecord(bt->done, st);
    if (e == hipSuccess) bt->launched = true;
    return after_launch(e, st, "batch launch");
}

sympix_status sympix_batch_tune(sympix_batch *bt, void *stream, int32_t *chosen, double *ms_out) {
    if (!bt) return fail(SYMPIX_EINVAL, "NULL batch");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    double best_ms = 0.0;
    int32_t best = -1;
    sympix_status s = SYMPIX_OK;
    for (int32_t c = 0; c < SYMPIX_NSCHED * SYMPIX_NTILINGS && s == SYMPIX_OK; ++c) {
        s = capture_batch(bt, c % SYMPIX_NSCHED, c / SYMPIX_NSCHED);
        if (s != SYMPIX_OK) break;
        e = hipGraphLaunch(bt->exec, st);                       // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = hipGraphLaunch(bt->exec, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventRecord(bt->done, st);
        if (e == hipSuccess) bt->launched = true;
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            s = hip_fail(e, "timing a batch schedule");
            break;
        }
        if (ms_out) ms_out[c] = ms;
        if (best < 0 || ms < best_ms) {
            best = c;
            best_ms = ms;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s != SYMPIX_OK) return s;
    s = capture_batch(bt, best % SYMPIX_NSCHED, best / SYMPIX_NSCHED);
    if (s != SYMPIX_OK) return s;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[bt->shape] = best;
        const std::string path = tune_cache_file();
        if (!path.empty() && !write_tune_file(path, bt->shape, best))
            return fail(SYMPIX_EINVAL, "could not write the tuner cache file " + path);
    }
    if (chosen) *chosen = best;
    return SYMPIX_OK;
}

sympix_status sympix_batch_plan(const sympix_batch *bt, int32_t *plan) {
    if (!bt || !plan) return fail(SYMPIX_EINVAL, "NULL argument");
    *plan = bt->schedule + SYMPIX_NSCHED * bt->tiling;
    return SYMPIX_OK;
}

void sympix_batch_destroy(sympix_batch *bt) {
    if (bt) free_batch(bt);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Two grids: B-hat = Y_2 B Y_1^T (Eqs. 13, 16) and B-hat^T N_2^-1 B-hat.
// ---------------------------------------------------------------------------
namespace {

// Device copies of a pair's tables: ring tables of g1 then g2, unique-block
// descriptors, class tables of the contraction, and the B-hat expansion list.
struct DevCross {
    double *ring_theta = nullptr;
    double *ring_sin = nullptr;
    UInfo *uinfo = nullptr;
    sympix::DevClass *classes = nullptr;
    int32_t *class_terms = nullptr;
    int32_t *class_blk = nullptr;
    int32_t *class_itab = nullptr;
    int32_t *gtiles = nullptr;          // dispatch table of the class-grid launch
    int32_t *exp_items = nullptr;
    int32_t *exp_blk = nullptr;
};

void free_dev_cross(DevCross &d) {
    hipFree(d.ring_theta);
    hipFree(d.ring_sin);
    hipFree(d.uinfo);
    hipFree(d.classes);
    hipFree(d.class_terms);
    hipFree(d.class_blk);
    hipFree(d.class_itab);
    hipFree(d.gtiles);
    hipFree(d.exp_items);
    hipFree(d.exp_blk);
    d = DevCross();
}

}  // namespace

struct sympix_cross {
    const sympix_grid *g2 = nullptr;      // auxiliary grid: rows of B-hat, N_2^-1
    const sympix_grid *g1 = nullptr;      // grid of the unknowns: columns, stored blocks
    sympix::CrossGeometry x;
    mutable std::mutex mu;
    mutable std::map<int, DevCross> dev;
};

namespace {

sympix_status cross_tables(const sympix_cross *c, int device, const DevCross **out) {
    std::lock_guard<std::mutex> lock(c->mu);
    auto it = c->dev.find(device);
    if (it != c->dev.end()) {
        *out = &it->second;
        return SYMPIX_OK;
    }
    const Geometry &g1 = c->g1->geo, &g2 = c->g2->geo;
    const sympix::CrossGeometry &x = c->x;
    std::vector<double> th(g1.theta), sn(g1.sin_theta);
    th.insert(th.end(), g2.theta.begin(), g2.theta.end());
    sn.insert(sn.end(), g2.sin_theta.begin(), g2.sin_theta.end());
    std::vector<UInfo> uinfo(x.nunique());
    for (int64_t u = 0; u < x.nunique(); ++u) {
        const int64_t I = x.rep_i[u], J = x.rep_j[u];
        const int bI = g2.tile_band[I], bJ = g1.tile_band[J];
        UInfo f;
        f.ring0_i = g1.nrings + g2.band_ring0[bI];   // rows: rings of g2, after those of g1
        f.ring0_j = g1.band_ring0[bJ];
        f.n_i = g2.k * g2.band_tiles[bI];
        f.n_j = g1.k * g1.band_tiles[bJ];
        f.p0_i = (int32_t)((I - g2.band_tile0[bI]) * g2.k);
        f.p0_j = (int32_t)((J - g1.band_tile0[bJ]) * g1.k);
        f.pad0 = f.pad1 = 0;
        uinfo[u] = f;
    }
    DevCross d;
    hipError_t e = upload(&d.ring_theta, th.data(), th.size());
    if (e == hipSuccess) e = upload(&d.ring_sin, sn.data(), sn.size());
    if (e == hipSuccess) e = upload(&d.uinfo, uinfo.data(), uinfo.size());
    if (e == hipSuccess)
        e = upload(&d.classes, reinterpret_cast<const sympix::DevClass *>(x.cls.classes.data()), x.cls.classes.size());
    if (e == hipSuccess) e = upload(&d.class_terms, x.cls.class_terms.data(), x.cls.class_terms.size());
    if (e == hipSuccess) e = upload(&d.class_blk, x.cls.class_blk.data(), x.cls.class_blk.size());
    if (e == hipSuccess) e = upload(&d.class_itab, x.cls.class_itab.data(), x.cls.class_itab.size());
    if (e == hipSuccess) e = upload(&d.gtiles, x.cls.gtiles.data(), x.cls.gtiles.size());
    if (e == hipSuccess) e = upload(&d.exp_items, x.exp_items.data(), x.exp_items.size());
    if (e == hipSuccess) e = upload(&d.exp_blk, x.exp_blk.data(), x.exp_blk.size());
    if (e != hipSuccess) {
        free_dev_cross(d);
        return e == hipErrorOutOfMemory ? fail(SYMPIX_ENOMEM, "device allocation for the two-grid tables failed")
                                        : hip_fail(e, "uploading the two-grid tables");
    }
    auto res = c->dev.emplace(device, d);
    *out = &res.first->second;
    return SYMPIX_OK;
}

sympix_status check_cross_kernel(const sympix_cross *c, const sympix_kernel *kr) {
    if (!c || !kr) return fail(SYMPIX_EINVAL, "NULL pair or kernel");
    if (kr->x != c) return fail(SYMPIX_EINVAL, "kernel was not tabulated for this pair of grids");
    if (c->g1->geo.k != 8) return fail(SYMPIX_EUNSUPPORTED, "device sampling is implemented for k = 8 only");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != kr->device) return fail(SYMPIX_EINVAL, "kernel lives on another device than the current one");
    return SYMPIX_OK;
}

}  // namespace

extern "C" {

sympix_status sympix_cross_create(const sympix_grid *g2, const sympix_grid *g1, sympix_cross **out) {
    if (!out) return fail(SYMPIX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g2 || !g1) return fail(SYMPIX_EINVAL, "NULL grid");
    sympix_cross *c = injected_alloc_failure() ? nullptr : new (std::nothrow) sympix_cross();
    if (!c) return fail(SYMPIX_ENOMEM, "host allocation failed");
    c->g2 = g2;
    c->g1 = g1;
    std::string err;
    const int rc = injected_alloc_failure() ? (err = "host allocation failed building the two-grid tables (injected)", -3)
                                            : sympix::build_cross(g2->geo, g1->geo, c->x, err);
    if (rc != 0) {
        delete c;
        return fail((sympix_status)rc, err);
    }
    *out = c;
    return SYMPIX_OK;
}

void sympix_cross_destroy(sympix_cross *c) {
    if (!c) return;
    for (auto &kv : c->dev) free_dev_cross(kv.second);
    delete c;
}

sympix_status sympix_cross_dims(const sympix_cross *c, sympix_cross_sizes *out) {
    if (!c || !out) return fail(SYMPIX_EINVAL, "NULL argument");
    const sympix::CrossGeometry &x = c->x;
    out->lmax_eff = x.lmax_eff;
    out->max_terms = x.cls.max_class_terms;
    out->nadjacency = (int64_t)x.adj_col.size();
    out->nunique = x.nunique();
    out->nblocks = c->g1->geo.nblocks();
    out->nterms = (int64_t)x.terms.size();
    out->y_pattern_max = x.y_pattern_max;
    return SYMPIX_OK;
}

sympix_status sympix_cross_neighbours(const sympix_cross *c, int32_t *container, int64_t *row_ptr, int32_t *col,
                                      int32_t *uid) {
    if (!c) return fail(SYMPIX_EINVAL, "NULL pair");
    const sympix::CrossGeometry &x = c->x;
    if (container) std::memcpy(container, x.container.data(), x.container.size() * sizeof(int32_t));
    if (row_ptr) std::memcpy(row_ptr, x.adj_ptr.data(), x.adj_ptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, x.adj_col.data(), x.adj_col.size() * sizeof(int32_t));
    if (uid) std::memcpy(uid, x.adj_uid.data(), x.adj_uid.size() * sizeof(int32_t));
    return SYMPIX_OK;
}

sympix_status sympix_cross_unique(const sympix_cross *c, int32_t *key_band_i, int32_t *key_band_j,
                                  int64_t *key_delta) {
    if (!c) return fail(SYMPIX_EINVAL, "NULL pair");
    const sympix::CrossGeometry &x = c->x;
    if (key_band_i) std::memcpy(key_band_i, x.key_band_i.data(), x.key_band_i.size() * sizeof(int32_t));
    if (key_band_j) std::memcpy(key_band_j, x.key_band_j.data(), x.key_band_j.size() * sizeof(int32_t));
    if (key_delta) std::memcpy(key_delta, x.key_delta.data(), x.key_delta.size() * sizeof(int64_t));
    return SYMPIX_OK;
}

sympix_status sympix_kernel_tabulate_cross(const sympix_cross *c, const double *coef_l, int32_t ncoef,
                                           double radius, int32_t n_nodes, void *stream, sympix_kernel **out) {
    if (!out) return fail(SYMPIX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !coef_l) return fail(SYMPIX_EINVAL, "NULL pair or coefficients");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const DevCross *dx = nullptr;
    sympix_status s = cross_tables(c, device, &dx);
    if (s != SYMPIX_OK) return s;
    TabSource src{c->x.lmax_eff, c->x.y_pattern_max, c->x.nunique(), dx->uinfo, dx->ring_theta, dx->ring_sin};
    return tabulate(src, nullptr, c, device, coef_l, ncoef, radius, n_nodes, (hipStream_t)stream, out);
}

sympix_status sympix_sample_B_cross(const sympix_cross *c, const sympix_kernel *b, double *out_dev, int64_t out_len,
                                    void *stream) {
    sympix_status s = check_cross_kernel(c, b);
    if (s != SYMPIX_OK) return s;
    const sympix::CrossGeometry &x = c->x;
    if (out_len != (int64_t)x.adj_col.size() * sympix::kBlockElems)
        return fail(SYMPIX_ESIZE, "out_len must be nadjacency * k^4");
    if (out_len > 0 && !out_dev) return fail(SYMPIX_EINVAL, "out_dev is NULL");
    if (((uintptr_t)out_dev) % 16) return fail(SYMPIX_EINVAL, "out_dev must be 16-byte aligned");
    const DevCross *dx = nullptr;
    s = cross_tables(c, b->device, &dx);
    if (s != SYMPIX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return after_launch(sympix::launch_expand(b->u64, dx->exp_items, (int64_t)x.exp_items.size() / 4, dx->exp_blk,
                                              out_dev, st),
                        st, "sample_B_cross");
}

sympix_status sympix_sample_BtNB_cross(const sympix_cross *c, const sympix_kernel *b, const double *ninv2_dev,
                                       int64_t ninv2_len, int32_t prec, double *out_dev, int64_t out_len,
                                       void *stream) {
    sympix_status s = check_cross_kernel(c, b);
    if (s != SYMPIX_OK) return s;
    const Geometry &g1 = c->g1->geo, &g2 = c->g2->geo;
    const sympix::CrossGeometry &x = c->x;
    if (prec < SYMPIX_FP64 || prec > SYMPIX_BF16X6) return fail(SYMPIX_EINVAL, "unknown precision mode");
    if (ninv2_len != g2.npix) return fail(SYMPIX_ESIZE, "ninv2_len must be npix of the auxiliary grid");
    const int64_t nblocks = g1.nblocks();
    if (out_len != nblocks * sympix::kBlockElems) return fail(SYMPIX_ESIZE, "out_len must be nblocks * k^4");
    if ((g2.npix > 0 && !ninv2_dev) || (out_len > 0 && !out_dev)) return fail(SYMPIX_EINVAL, "NULL device buffer");
    if (((uintptr_t)out_dev) % 16 || ((uintptr_t)ninv2_dev) % 32)
        return fail(SYMPIX_EINVAL, "out_dev must be 16-byte and ninv2_dev 32-byte aligned");
    if (out_len > 0) {
        const char *o = (const char *)out_dev, *w = (const char *)ninv2_dev;
        const size_t ob = (size_t)out_len * sizeof(double), nb = (size_t)ninv2_len * sizeof(double);
        if (o < w + nb && w < o + ob) return fail(SYMPIX_EINVAL, "the output overlaps ninv2_dev");
    }
    if (x.cls.max_class_terms > sympix::kMaxClassTerms)
        return fail(SYMPIX_EUNSUPPORTED, "a block has more contraction tiles than the class GEMM supports");
    const DevCross *dx = nullptr;
    s = cross_tables(c, b->device, &dx);
    if (s != SYMPIX_OK) return s;
    sympix::BtnbArgs a;
    a.u64t = b->u64t;
    a.ut32 = b->ut32;
    a.classes = dx->classes;
    a.class_terms = dx->class_terms;
    a.class_blk = dx->class_blk;
    a.class_itab = dx->class_itab;
    a.mtiles = dx->gtiles;
    a.nmtiles = (int64_t)x.cls.gtiles.size() / 4;
    a.nblocks = nblocks;
    a.npix = g2.npix;
    a.ninv = ninv2_dev;
    a.out = out_dev;
    a.du64 = nullptr;
    a.blk_uid = nullptr;
    a.outD = nullptr;
    return launch_contraction(a, b->device, prec, false, (hipStream_t)stream, "sample_BtNB_cross");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Spherical harmonic transforms on the SymPix geometry (Eq. 1) and the
// degrade of Eq. 14.
// ---------------------------------------------------------------------------
struct sympix_sht {
    const sympix_grid *g = nullptr;
    int32_t lmax = 0;
    int device = 0;
    sympix::ShtDesc d{};
    double *fbuf = nullptr;      // nrings (L+1) 2: Legendre <-> Fourier stage
    double *ac = nullptr;        // m-major cos coefficients
    double *as = nullptr;        // m-major sin coefficients
    void *block = nullptr;       // one allocation holding the tables and buffers
};

namespace {

// FFT passes of a ring of n = 2^a 3^b 5^c pixels: radix 4 first, then 2, 3, 5
bool ring_radices(int32_t n, int8_t out[16]) {
    int np = 0;
    for (int r : {4, 2, 3, 5})
        while (n % r == 0 && np < 15) {
            out[1 + np++] = (int8_t)r;
            n /= r;
        }
    out[0] = (int8_t)np;
    return n == 1;
}

sympix_status sht_check(const sympix_sht *s, const void *in, int64_t in_len, int64_t want_in, const void *out,
                        int64_t out_len, int64_t want_out) {
    if (!s) return fail(SYMPIX_EINVAL, "NULL plan");
    if (in_len != want_in || out_len != want_out) return fail(SYMPIX_ESIZE, "buffer length does not match the plan");
    if ((want_in > 0 && !in) || (want_out > 0 && !out)) return fail(SYMPIX_EINVAL, "NULL device buffer");
    if (((uintptr_t)in) % 8 || ((uintptr_t)out) % 8) return fail(SYMPIX_EINVAL, "buffers must be 8-byte aligned");
    const char *a = (const char *)in, *b = (const char *)out;
    if (a < b + out_len * 8 && b < a + in_len * 8) return fail(SYMPIX_EINVAL, "input and output overlap");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != s->device)
        return fail(SYMPIX_EINVAL, "the plan lives on another device");
    return SYMPIX_OK;
}

}  // namespace

extern "C" {

sympix_status sympix_sht_create(const sympix_grid *g, int32_t lmax_sh, sympix_sht **out) {
    if (!g || !out) return fail(SYMPIX_EINVAL, "NULL argument");
    *out = nullptr;
    if (lmax_sh < 0) return fail(SYMPIX_EINVAL, "lmax_sh must be >= 0");
    if (lmax_sh > sympix::kShtMaxL) return fail(SYMPIX_EUNSUPPORTED, "lmax_sh above 4095");
    const Geometry &geo = g->geo;
    const int32_t L = lmax_sh, nr = geo.nrings, nh = nr / 2, k = geo.k;
    // ring tables: band of each ring, its length, first pixel and weight
    std::vector<int32_t> rn(nr, 0);
    std::vector<int64_t> pix0(nr, 0);
    std::vector<double> rw(nr, 0.0);
    std::vector<int8_t> rad((size_t)nr * 16, 0);
    int32_t max_ring = 0, max_fft = 0;
    for (size_t b = 0; b < geo.band_tiles.size(); ++b) {
        const int32_t n = k * geo.band_tiles[b];
        for (int32_t r = 0; r < k; ++r) {
            const int32_t j = geo.band_ring0[b] + r;
            rn[j] = n;
            pix0[j] = geo.band_tile0[b] * (int64_t)k * k + r;
            rw[j] = geo.weight[j] * 2.0 * kPi / (double)n;
            // an even ring takes an FFT of half its length (its values paired as complex)
            if (!ring_radices(n % 2 == 0 ? n / 2 : n, &rad[(size_t)j * 16]))
                return fail(SYMPIX_EUNSUPPORTED, "a ring length is not of the form 2^a 3^b 5^c");
        }
        max_ring = std::max(max_ring, n);
        max_fft = std::max(max_fft, n % 2 == 0 ? n / 2 : n);
    }
    if (max_ring > sympix::kShtMaxRing) return fail(SYMPIX_EUNSUPPORTED, "a ring is longer than 8192 pixels");
    if (nh > sympix::kShtMaxHalfRings) return fail(SYMPIX_EUNSUPPORTED, "more than 4096 rings");
    // lambda_mm of the northern rings: the product recurrence lambda_mm =
    // lambda_{m-1,m-1} sqrt((2m+1)/(2m)) sin(theta) from 1/sqrt(4 pi), kept as
    // mant * 2^exp with mant >= 2^-300
    std::vector<double> mant((size_t)(L + 1) * nh), ring_cos(nh);
    std::vector<int32_t> ex((size_t)(L + 1) * nh);
    for (int32_t r = 0; r < nh; ++r) {
        ring_cos[r] = geo.cos_theta[r];
        const double st = geo.sin_theta[r];
        double v = 1.0 / std::sqrt(4.0 * kPi);
        int32_t e = 0;
        for (int32_t m = 0; m <= L; ++m) {
            if (m > 0) {
                v *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * st;
                if (v < 0x1p-300) {
                    v *= 0x1p300;
                    e -= 300;
                }
            }
            mant[(size_t)m * nh + r] = v;
            ex[(size_t)m * nh + r] = e;
        }
    }
    // m-major rows and the monic recurrence's per-degree values (the same
    // for every ring): b_i = ((l-1)^2 - m^2) / (4 (l-1)^2 - 1), b_0 = -1, and
    // K_i = prod alpha_j over j in [64 floor(i / 64), i], j >= 1, alpha_j^2 =
    // (4 l_j^2 - 1) / (l_j^2 - m^2); products and quotients in long double
    std::vector<int64_t> row_off(L + 1);
    int64_t nrow = 0;
    for (int32_t m = 0; m <= L; ++m) {
        row_off[m] = nrow;
        nrow += ((int64_t)(L - m + 1) + sympix::kShtRowPad + 3) / 4 * 4;
    }
    std::vector<double> rec_b((size_t)nrow, 0.0), rec_k((size_t)nrow, 0.0);
    for (int32_t m = 0; m <= L; ++m) {
        double *bb = &rec_b[(size_t)row_off[m]], *kk = &rec_k[(size_t)row_off[m]];
        const long double mm = (long double)m * m;
        long double k2 = 1.0L;
        for (int32_t i = 0; i <= L - m; ++i) {
            const long double l = (long double)(m + i), l1 = l - 1.0L;
            bb[i] = i == 0 ? -1.0 : (double)((l1 * l1 - mm) / (4.0L * l1 * l1 - 1.0L));
            const long double a2 = i == 0 ? 1.0L : (4.0L * l * l - 1.0L) / (l * l - mm);
            k2 = (i % 64 == 0) ? a2 : k2 * a2;
            kk[i] = (double)std::sqrt(k2);
        }
    }
    sympix_sht *s = injected_alloc_failure() ? nullptr : new (std::nothrow) sympix_sht();
    if (!s) return fail(SYMPIX_ENOMEM, "host allocation failed");
    s->g = g;
    s->lmax = L;
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipGetDevice");
    }
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t o = 0;
    const size_t o_cos = o;   o += up(sizeof(double) * nh);
    const size_t o_mant = o;  o += up(sizeof(double) * mant.size());
    const size_t o_exp = o;   o += up(sizeof(int32_t) * ex.size());
    const size_t o_n = o;     o += up(sizeof(int32_t) * nr);
    const size_t o_pix = o;   o += up(sizeof(int64_t) * nr);
    const size_t o_w = o;     o += up(sizeof(double) * nr);
    const size_t o_rad = o;   o += up(rad.size());
    const size_t o_f = o;     o += up(sizeof(double) * 2 * (size_t)nr * (L + 1));
    const size_t o_row = o;   o += up(sizeof(int64_t) * (L + 1));
    const size_t o_b = o;     o += up(sizeof(double) * (size_t)nrow);
    const size_t o_k = o;     o += up(sizeof(double) * (size_t)nrow);
    const size_t o_ac = o;    o += up(sizeof(double) * (size_t)nrow);
    const size_t o_as = o;    o += up(sizeof(double) * (size_t)nrow);
    e = injected_alloc_failure() ? hipErrorOutOfMemory : hipMalloc(&s->block, o);
    if (e != hipSuccess) {
        s->block = nullptr;
        delete s;
        return e == hipErrorOutOfMemory ? fail(SYMPIX_ENOMEM, "device allocation for the transform plan failed")
                                        : hip_fail(e, "hipMalloc");
    }
    char *base = (char *)s->block;
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(base + off, src, bytes, hipMemcpyHostToDevice);
    };
    put(o_cos, ring_cos.data(), sizeof(double) * nh);
    put(o_mant, mant.data(), sizeof(double) * mant.size());
    put(o_exp, ex.data(), sizeof(int32_t) * ex.size());
    put(o_n, rn.data(), sizeof(int32_t) * nr);
    put(o_pix, pix0.data(), sizeof(int64_t) * nr);
    put(o_w, rw.data(), sizeof(double) * nr);
    put(o_rad, rad.data(), rad.size());
    put(o_row, row_off.data(), sizeof(int64_t) * (L + 1));
    put(o_b, rec_b.data(), sizeof(double) * (size_t)nrow);
    put(o_k, rec_k.data(), sizeof(double) * (size_t)nrow);
    // the rows' padding of ac / as stays zero: the kernels write entries i <= L - m only
    if (e == hipSuccess) e = hipMemset(base + o_ac, 0, (o_as - o_ac) + sizeof(double) * (size_t)nrow);
    if (e == hipSuccess) e = sympix::sht_prepare(max_fft);
    if (e != hipSuccess) {
        hipFree(s->block);
        delete s;
        return hip_fail(e, "uploading the transform plan");
    }
    sympix::ShtDesc &d = s->d;
    d.lmax = L;
    d.nrings = nr;
    d.nhalf = nh;
    d.k = k;
    d.max_ring = max_ring;
    d.max_fft = max_fft;
    d.ring_cos = (const double *)(base + o_cos);
    d.lmm_mant = (const double *)(base + o_mant);
    d.lmm_exp = (const int32_t *)(base + o_exp);
    d.ring_n = (const int32_t *)(base + o_n);
    d.ring_pix0 = (const int64_t *)(base + o_pix);
    d.ring_w = (const double *)(base + o_w);
    d.ring_rad = (const int8_t *)(base + o_rad);
    d.row_off = (const int64_t *)(base + o_row);
    d.rec_b = (const double *)(base + o_b);
    d.rec_k = (const double *)(base + o_k);
    s->fbuf = (double *)(base + o_f);
    s->ac = (double *)(base + o_ac);
    s->as = (double *)(base + o_as);
    *out = s;
    return SYMPIX_OK;
}

void sympix_sht_destroy(sympix_sht *s) {
    if (!s) return;
    hipFree(s->block);
    delete s;
}

sympix_status sympix_sht_synthesis(sympix_sht *s, const double *alm_dev, int64_t alm_len, double *map_dev,
                                   int64_t map_len, void *stream) {
    if (!s) return fail(SYMPIX_EINVAL, "NULL plan");
    const int64_t nalm = (int64_t)(s->lmax + 1) * (s->lmax + 1);
    sympix_status st = sht_check(s, alm_dev, alm_len, nalm, map_dev, map_len, s->g->geo.npix);
    if (st != SYMPIX_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    return after_launch(sympix::sht_synthesis(s->d, alm_dev, s->ac, s->as, s->fbuf, map_dev, false, hs), hs,
                        "sht_synthesis");
}

static sympix_status sht_transpose(sympix_sht *s, const double *map_dev, int64_t map_len, double *alm_dev,
                                   int64_t alm_len, void *stream, bool weighted, const char *what) {
    if (!s) return fail(SYMPIX_EINVAL, "NULL plan");
    const int64_t nalm = (int64_t)(s->lmax + 1) * (s->lmax + 1);
    sympix_status st = sht_check(s, map_dev, map_len, s->g->geo.npix, alm_dev, alm_len, nalm);
    if (st != SYMPIX_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    return after_launch(sympix::sht_adjoint(s->d, map_dev, s->fbuf, s->ac, s->as, alm_dev, weighted, hs), hs, what);
}

sympix_status sympix_sht_adjoint(sympix_sht *s, const double *map_dev, int64_t map_len, double *alm_dev,
                                 int64_t alm_len, void *stream) {
    return sht_transpose(s, map_dev, map_len, alm_dev, alm_len, stream, false, "sht_adjoint");
}

sympix_status sympix_sht_analysis(sympix_sht *s, const double *map_dev, int64_t map_len, double *alm_dev,
                                  int64_t alm_len, void *stream) {
    return sht_transpose(s, map_dev, map_len, alm_dev, alm_len, stream, true, "sht_analysis");
}

sympix_status sympix_sht_degrade(sympix_sht *obs, sympix_sht *target, const double *theta_obs_dev,
                                 int64_t obs_len, double *theta2_dev, int64_t target_len, void *stream) {
    if (!obs || !target) return fail(SYMPIX_EINVAL, "NULL plan");
    if (obs->lmax != target->lmax) return fail(SYMPIX_EINVAL, "the two plans have different band limits");
    if (obs->device != target->device) return fail(SYMPIX_EINVAL, "the two plans live on different devices");
    sympix_status st = sht_check(obs, theta_obs_dev, obs_len, obs->g->geo.npix, theta2_dev, target_len,
                                 target->g->geo.npix);
    if (st != SYMPIX_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    // Y_obs^T theta into the observation plan's m-major buffers, then W_2 Y_2
    // of them on the target grid
    hipError_t e = sympix::sht_adjoint(obs->d, theta_obs_dev, obs->fbuf, obs->ac, obs->as, nullptr, false, hs);
    if (e == hipSuccess)
        e = sympix::sht_synthesis(target->d, nullptr, obs->ac, obs->as, target->fbuf, theta2_dev, true, hs);
    return after_launch(e, hs, "sht_degrade");
}

}  // extern "C"
