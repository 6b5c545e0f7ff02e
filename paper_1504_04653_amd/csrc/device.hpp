// Device-side data layouts and launch functions (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "geometry.hpp"

namespace sympix {

// Geometry of one unique block: rows are the k^2 pixels of a representative
// tile I, columns those of tile J.  Ring of local pixel (c, r) is ring0 + r,
// its index on the ring is p0 + c, the ring holds n pixels.
struct UInfo {
    int32_t ring0_i, ring0_j;
    int32_t n_i, n_j;
    int32_t p0_i, p0_j;
    int32_t pad0, pad1;
};

// A class of stored blocks sharing their contraction pattern (see geometry.hpp).
struct DevClass {
    int32_t nterms, nblocks, term0, blk0;
    int64_t itab0;
    int32_t sym, pad;      // sym: every member block is symmetric
};

// Tabulated kernel as seen by device code.
struct KTable {
    const double *table;  // n_nodes values, node i at s = |i - 1| h
    int32_t n_nodes;
    double inv_h;
    double y_cut;         // values at y > y_cut are 0 (+inf: no cut)
};

constexpr int kBlockDim = 64;              // k^2 for k = 8
constexpr int kBlockElems = 64 * 64;
constexpr int kMaxClassTerms = 128;     // contraction terms a class may have (two-grid blocks have up to ~4x
                                        // the one-grid count when Y_2 has twice Y_1's resolution)
constexpr int kTileStride = kMaxClassTerms + 1;   // LDS row stride of the member-tile table (odd: no bank
                                                  // conflicts when the lanes of a wave read 16 rows)

// a6: table of sum_l c_l P_l(1 - s^2), c_l = (2l+1) coef_l / 4 pi
hipError_t launch_tabulate(const double *coef, int32_t lmax, double h, double *table,
                           int32_t n_nodes, hipStream_t st);
// evaluation of the table at arbitrary y (tests of the interpolation)
hipError_t launch_eval(KTable kt, const double *y, double *out, int64_t n, hipStream_t st);
// a7: every unique block, FP64 row-major [uid][p][q] plus FP64 and FP32
// copies transposed [uid][q][p]
hipError_t launch_unique_eval(KTable kt, const UInfo *uinfo, int64_t nunique, const double *ring_theta,
                              const double *ring_sin, double *u64, double *u64t, float *ut32, hipStream_t st);
// a8: D-hat expansion: each work item {uid, first, count, 0} copies unique
// block uid into the stored blocks exp_blk[first .. first + count)
hipError_t launch_expand(const double *u64, const int32_t *items, int64_t nitems, const int32_t *exp_blk,
                         double *out, hipStream_t st);
// pixel-domain convolution g = B-hat f over chunks of kConvTiles output tiles
hipError_t launch_convolve(const double *u64, const int32_t *chunks, int64_t nchunks, const int32_t *slots,
                           const double *f, double *g, hipStream_t st);
// a9: B-hat^T N^-1 B-hat contraction
struct BtnbArgs {
    const double *u64t;
    const float *ut32;
    const DevClass *classes;
    const int32_t *class_terms, *class_blk, *class_itab;
    const int32_t *mtiles;    // the class-grid dispatch table: one slot per workgroup,
    int64_t nmtiles;          // 4 ints as a member tile, groups 0 an empty slot
    uint16_t *wsplit[3];      // scratch: N^-1 split into BF16 parts, npix each
    float *wf32;              // scratch: N^-1 rounded to FP32, npix
    int64_t npix;
    int64_t nblocks;
    const double *ninv;
    double *out;
    // optional D-hat blocks written by the same launch:
    // stored block n gets unique block blk_uid[n] of du64 (row-major FP64)
    const double *du64;
    const int32_t *blk_uid;
    double *outD;             // nullptr: B-hat^T N^-1 B-hat only
};
hipError_t launch_btnb(int prec, const BtnbArgs &a, hipStream_t st);

// Operands of the FP64 class GEMM (device pointers).
struct ProblemDesc64 {
    const int32_t *mtiles;
    const DevClass *classes;
    const int32_t *cterms, *cblk, *citab;
    const double *u64t;
    const double *w;          // N^-1
    double *out;
    const double *du64;       // D-hat: unique blocks, row-major FP64 (with outD)
    const int32_t *blk_uid;   // unique block of each stored block
    double *outD;             // D-hat output, or nullptr
};

// Operands of the split-BF16 class GEMM (device pointers).
struct ProblemDescB {
    const int32_t *mtiles;
    const DevClass *classes;
    const int32_t *cterms, *cblk, *citab;
    const float *ut32;
    const uint16_t *w[3];     // N^-1 split into BF16 parts
    double *out;
    const double *du64;       // D-hat: unique blocks, row-major FP64 (with outD)
    const int32_t *blk_uid;   // unique block of each stored block
    double *outD;             // D-hat output, or nullptr
};

// Operands of the FP32 class GEMM for one problem (device pointers).
struct ProblemDesc {
    const int32_t *mtiles;
    const DevClass *classes;
    const int32_t *cterms, *cblk, *citab;
    const float *ut32;
    float *wf;                // N^-1 rounded to FP32 (written by the launch)
    double *out;
    const double *du64;       // D-hat: unique blocks, row-major FP64 (with outD)
    const int32_t *blk_uid;   // unique block of each stored block
    double *outD;             // D-hat output, or nullptr
};

// a10: one batched launch.  host_desc / host_descb / host_desc64 / ninv /
// npix / gtiles / ngtiles / wsplit are host arrays of nprob entries (wsplit: 3
// per problem; gtiles: device pointers to each problem's class-grid dispatch
// table of ngtiles slots, used by the one-launch-per-problem schedule in place
// of the descriptors' member tiles); desc, descb, desc64, items, qb and
// counters live on the device.
// prec: 0 FP64 (desc64, host_desc64; N^-1 read as given), 1 FP32 (desc,
// host_desc), 2 or 3 split BF16 with that many parts (descb, host_descb, and
// the N^-1 parts in wsplit).
struct BatchLaunch {
    int32_t nprob;
    int32_t prec;
    const ProblemDesc64 *host_desc64;
    const ProblemDesc64 *desc64;
    const ProblemDesc *host_desc;
    const ProblemDescB *host_descb;
    uint16_t *const *wsplit;
    const ProblemDescB *descb;
    const double *const *ninv;
    const int64_t *npix;
    const int32_t *const *gtiles;
    const int64_t *ngtiles;
    const ProblemDesc *desc;
    const int32_t *items;     // 2 per item: problem, member tile
    int64_t nitems;
    const int32_t *qb;        // nq + 1 queue bounds
    int32_t nq;
    int32_t *counters;        // nq
    bool persistent;          // false: one class-GEMM launch per problem
    int32_t nworkgroups;
};
hipError_t launch_batch(const BatchLaunch &b, hipStream_t st);

// The allocation-free sampling call keeps N^-1 in the MFMA operand format in a
// file-scope device array of 3 * kNoAllocMaxPix BF16 words (96 MiB): up to
// kNoAllocMaxPix pixels in every mode.  noalloc_scratch returns the array's
// address on `device`, which must be current (looked up once per device).
constexpr int64_t kNoAllocMaxPix = int64_t(1) << 24;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_scratch(int device, void **ptr);
hipError_t batch_occupancy(int prec, int *workgroups_per_cu);

}  // namespace sympix
