// HIP kernels for SymPix local-operator sampling on gfx950 (CDNA4, wave64).
//
//   k_tabulate     kernel table of Eq. 10, FP64 Legendre recurrence in y
//   k_eval         table lookups at arbitrary y (interpolation tests)
//   k_unique_eval  one workgroup per unique block (Section 2.3 symmetry keys):
//                  pair geometry, table lookup, radial cut; writes FP64
//                  row-major and FP64 / FP32 copies transposed via LDS
//   k_expand       D-hat: streams each stored block from its unique block
//   k_convolve     pixel-domain convolution g = B-hat f, one FP64 GEMM per
//                  unique block over 32 output tiles
//   k_class_f64    B-hat^T N^-1 B-hat (Eq. 15) in FP64 as one GEMM per class of
//                  blocks that share their contraction pattern; the class
//                  kernels' <true> instantiations also copy D-hat (combined call)
//   k_ninv_f32     N^-1 rounded to FP32
//   k_class_f32    FP32-MFMA contraction as one GEMM per class of blocks that
//                  share their contraction pattern, FP64 accumulation across tiles
//   k_batch_f64    the FP64 class GEMM of many problems in one persistent
//                  launch fed by per-XCD work queues
//   k_batch_f32    the same in FP32
//   k_split_ninv   N^-1 split into BF16 parts
//   k_class_bf16   the same GEMM in split BF16
//   k_batch_bf16   many problems in one persistent launch, split BF16
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "device.hpp"

namespace sympix {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Remap the workgroup index so that every XCD processes one contiguous range of
// the work list: neighbouring items share operands, which then stay in that
// XCD's L2.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_contiguous_index() {
    const int n = gridDim.x, b = blockIdx.x;
    const int x = b & 7, i = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + i;
}

// ---------------------------------------------------------------------------
// a6: kernel table.  Node i holds b at s = |i - 1| h, y = s^2 (node 0 mirrors
// node 2: the kernel is even in s).  Recurrence in y with D_l = P_l - P_{l-1}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tabulate(const double *__restrict__ coef, int lmax,
                                                  double h, double *__restrict__ table,
                                                  int n_nodes) {
    // Per-degree factors of the recurrence, staged in LDS a chunk of degrees
    // at a time by the whole workgroup: step l takes d <- A_l d - B_l y p with
    // A_l = l / (l + 1), B_l = (2l + 1) / (l + 1), then p <- p + d (now
    // P_{l+1}(1 - y)), and adds C_l p, C_l = (2l + 3) coef_{l+1} / 4 pi.
    constexpr int kChunk = 1024;
    __shared__ double sA[kChunk], sB[kChunk], sC[kChunk];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double s = (double)(i > 0 ? i - 1 : 1) * h;
    const double y = s * s;
    double p = 1.0;
    double acc = coef[0] * kInv4Pi;
    double d = 0.0;                      // step 0 gives d = -y (A_0 = 0, B_0 = 1)
    for (int l0 = 0; l0 < lmax; l0 += kChunk) {
        const int n = min(kChunk, lmax - l0);
        __syncthreads();                 // the previous chunk is used up
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const int l = l0 + t;
            sA[t] = (double)l / (double)(l + 1);
            sB[t] = (double)(2 * l + 1) / (double)(l + 1);
            sC[t] = (double)(2 * l + 3) * coef[l + 1] * kInv4Pi;
        }
        __syncthreads();
        for (int t = 0; t < n; ++t) {
            d = sA[t] * d - sB[t] * y * p;
            p = p + d;
            acc += sC[t] * p;
        }
    }
    if (i < n_nodes) table[i] = acc;
}

// 4-point Lagrange interpolation in s = sqrt(y) on nodes -1, 0, 1, 2 around
// the interval containing s; zero beyond the radial cut.
__device__ __forceinline__ double lookup(const KTable &kt, double y) {
    if (!(y <= kt.y_cut)) return 0.0;
    double u = sqrt(y) * kt.inv_h;
    u = fmin(u, (double)(kt.n_nodes - 3));
    int i = (int)u;
    i = min(i, kt.n_nodes - 4);
    const double t = u - (double)i;
    const double *T = kt.table + i;
    const double tp1 = t + 1.0, tm1 = t - 1.0, tm2 = t - 2.0;
    const double w0 = -t * tm1 * tm2 * (1.0 / 6.0);
    const double w1 = tp1 * tm1 * tm2 * 0.5;
    const double w2 = -tp1 * t * tm2 * 0.5;
    const double w3 = tp1 * t * tm1 * (1.0 / 6.0);
    return w0 * T[0] + w1 * T[1] + w2 * T[2] + w3 * T[3];
}

__global__ __launch_bounds__(256) void k_eval(KTable kt, const double *__restrict__ y,
                                              double *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = lookup(kt, y[i]);
}

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    __bf16 b = (__bf16)x;   // round to nearest even
    return __builtin_bit_cast(uint16_t, b);
}

__device__ __forceinline__ float bf16_value(uint16_t b) {
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// ---------------------------------------------------------------------------
// a7: unique blocks.  Element (p, q): row pixel p = c*8 + r of tile I, column
// pixel q of tile J.  dphi = pi N / (n_i n_j) with N reduced exactly into
// (-n_i n_j, n_i n_j]; y = 2 [sin^2(dtheta/2) + sin th1 sin th2 sin^2(dphi/2)].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_unique_eval(KTable kt, const UInfo *__restrict__ uinfo,
                                                     const double *__restrict__ ring_theta,
                                                     const double *__restrict__ ring_sin,
                                                     double *__restrict__ u64,
                                                     double *__restrict__ u64t,
                                                     float *__restrict__ ut32) {
    __shared__ double tile[64][65];
    const int64_t uid = blockIdx.x;
    const UInfo inf = uinfo[uid];
    const int64_t M = (int64_t)inf.n_i * inf.n_j;
    const double inv2M = 1.0 / (double)(2 * M);
    double *dst = u64 + uid * kBlockElems;
    for (int e = threadIdx.x; e < kBlockElems; e += 256) {
        const int p = e >> 6, q = e & 63;
        const int c = p >> 3, r = p & 7, c2 = q >> 3, r2 = q & 7;
        const int j1 = inf.ring0_i + r, j2 = inf.ring0_j + r2;
        int64_t N = (int64_t)(2 * (inf.p0_j + c2) + 1) * inf.n_i -
                    (int64_t)(2 * (inf.p0_i + c) + 1) * inf.n_j;
        while (N > M) N -= 2 * M;
        while (N <= -M) N += 2 * M;
        const double sp = sinpi((double)N * inv2M);               // sin(dphi / 2)
        const double sd = sin(0.5 * (ring_theta[j1] - ring_theta[j2]));
        const double y = 2.0 * (sd * sd + ring_sin[j1] * ring_sin[j2] * (sp * sp));
        const double v = lookup(kt, y);
        dst[e] = v;
        tile[p][q] = v;
    }
    __syncthreads();
    const int64_t base = uid * kBlockElems;
    for (int e = threadIdx.x; e < kBlockElems; e += 256) {
        const int q = e >> 6, p = e & 63;   // transposed layout [q][p]
        const double v = tile[p][q];
        u64t[base + e] = v;
        ut32[base + e] = (float)v;
    }
}

// ---------------------------------------------------------------------------
// a8: D-hat expansion.  Each stored block is a 32 KiB copy of its unique block.
// A workgroup holds one unique block in registers (8 x 16 bytes per thread)
// and writes it to up to 64 stored blocks with 16-byte non-temporal stores,
// so the unique blocks are read once and the kernel only streams writes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_expand(const double *__restrict__ u64,
                                                const int32_t *__restrict__ items,
                                                const int32_t *__restrict__ exp_blk,
                                                double *__restrict__ out) {
    const int32_t uid = items[4 * blockIdx.x], first = items[4 * blockIdx.x + 1];
    const int32_t count = items[4 * blockIdx.x + 2];
    const doublex2 *src = (const doublex2 *)(u64 + (int64_t)uid * kBlockElems);
    doublex2 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = src[threadIdx.x + 256 * j];
    for (int n = 0; n < count; ++n) {
        doublex2 *dst = (doublex2 *)(out + (int64_t)exp_blk[first + n] * kBlockElems);
#pragma unroll
        for (int j = 0; j < 8; ++j) __builtin_nontemporal_store(v[j], &dst[threadIdx.x + 256 * j]);
    }
}

// ---------------------------------------------------------------------------
// Pixel-domain convolution g = B-hat f (Section 4.1): g_J = sum_{K in nbr(J)}
// B_JK f_K.  One workgroup per chunk of kConvTiles (32) consecutive output
// tiles of a band, wave i computing output rows 16 i .. 16 i + 15 of all of
// them, as two 16-column MFMA tiles.  For every unique block u the chunk uses
// (a slot), one FP64 GEMM C += U_u F_u with C[p][j] the outputs of tile J0 + j
// and F_u[q][j] = f of the input tile that tile J0 + j multiplies with u
// (zero when it does not), so each unique block is read once per 32 tiles.
// F_u (32 tiles x 64 values) is loaded once by the workgroup into one of two
// LDS buffers, one barrier per slot; each wave loads only its own 16 rows of
// U_u.  Loads of the next slot go out before the current slot's MFMAs.  MFMA
// 16x16x4 FP64, MFMA m = 2 x + t with contraction index q = 8 x + 2 lk + t:
// lane (lr, lk) holds U[16 i + lr][q] and F[q][16 cg + lr]; its result holds
// rows 16 i + lk + 4 v of column 16 cg + lr.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_convolve(const double *__restrict__ u64, const int32_t *__restrict__ chunks,
                                                  const int32_t *__restrict__ slots, const double *__restrict__ f,
                                                  double *__restrict__ g) {
    constexpr int NT = kConvTiles, SW = 1 + kConvTiles;   // tiles per chunk, ints per slot
    constexpr int NCG = NT / 16, NFR = NT / 8;             // 16-column MFMA tiles, F chunks per thread
    static_assert(NT % 16 == 0 && NT <= 64, "16-column MFMA tiles, at most 64 KiB of staged F");
    // F of one slot: tile t's 64 values as 32 chunks of 16 bytes, chunk c at
    // 32 t + (c ^ (t & 15)), so each 16-lane read phase (16 tiles, one c)
    // touches 16 different bank groups
    __shared__ doublex2 sF[2][NT * 32];
    const int ch = xcd_contiguous_index();
    const int J0 = chunks[4 * ch], n = chunks[4 * ch + 1];
    const int s0 = chunks[4 * ch + 2], ns = chunks[4 * ch + 3];
    const int tid = threadIdx.x;
    const int i = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wave's rows 16 i .. 16 i + 15
    const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    // F staging: thread tid takes chunks tid + 256 r (r < NT / 8): tile (tid >> 5) + 8 r, chunk tid & 31
    const int ft = tid >> 5, fc = tid & 31;
    struct Ops { doublex2 a[8], fs[NFR]; };
    auto load = [&](int sl, Ops &o) {
        const int32_t *slot = slots + SW * (int64_t)(s0 + min(sl, ns - 1));
        const doublex2 *up = (const doublex2 *)(u64 + (int64_t)slot[0] * kBlockElems + (16 * i + lr) * 64 + 2 * lk);
#pragma unroll
        for (int x = 0; x < 8; ++x) o.a[x] = up[4 * x];   // the four lanes of a row read 64 contiguous bytes
#pragma unroll
        for (int r = 0; r < NFR; ++r) {
            const int K = slot[1 + ft + 8 * r];
            o.fs[r] = K >= 0 ? *(const doublex2 *)(f + (int64_t)K * 64 + 2 * fc) : doublex2{0.0, 0.0};
        }
    };
    auto stage = [&](const Ops &o, int buf) {
#pragma unroll
        for (int r = 0; r < NFR; ++r) {
            const int t = ft + 8 * r;
            sF[buf][32 * t + (fc ^ (t & 15))] = o.fs[r];
        }
    };
    doublex4 c[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) c[cg] = doublex4{0.0, 0.0, 0.0, 0.0};
    auto mfmas = [&](const Ops &o, int buf) {
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
            const int t = 16 * cg + lr;
#pragma unroll
            for (int x = 0; x < 8; ++x) {
                const doublex2 bf = sF[buf][32 * t + ((4 * x + lk) ^ (t & 15))];
                c[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[x][0], bf[0], c[cg], 0, 0, 0);
                c[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[x][1], bf[1], c[cg], 0, 0, 0);
            }
        }
    };
    Ops o0, o1;
    load(0, o0);
    stage(o0, 0);
    __syncthreads();
    // slot sl computes from buffer sl & 1 with its U rows in registers; the
    // next slot's loads go out first and its F is staged after the MFMAs
    for (int sl = 0; sl < ns; sl += 2) {
        load(sl + 1, o1);
        mfmas(o0, 0);
        stage(o1, 1);
        __syncthreads();
        if (sl + 1 >= ns) break;
        load(sl + 2, o0);
        mfmas(o1, 1);
        stage(o0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
        const int j = 16 * cg + lr;
        if (j < n) {
            double *o = g + (int64_t)(J0 + j) * 64 + 16 * i + lk;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[4 * v] = c[cg][v];
        }
    }
}

// ---------------------------------------------------------------------------
// D-hat copies made by a class-GEMM launch for the stored blocks of its tile
// (the combined call): each stored block gets its unique D-hat block
// (row-major FP64).  Chunk c of a tile is 16 bytes (c & 2047) of member row
// c >> 11; a wave's 64 chunks lie in one row, so the row is uniform.  Step stp
// of a workgroup of NT threads loads chunks [2 NT stp, 2 NT (stp + 1)), two per
// thread; they are stored one step later, right after that step's loads:
// stores and loads share one wait counter, and a store placed there is waited
// for only by the next step's operand wait.  sBlk[m] is the stored block of
// member row m (-1: none), sBlk[64 + m] its unique D-hat block.
// ---------------------------------------------------------------------------
struct DCopy {
    doublex2 v[2];
    double *dst[2];            // uniform: where the chunk row goes (nullptr: nowhere)
};

template <int NT>
__device__ __forceinline__ void dcopy_load(const double *__restrict__ du64, double *__restrict__ outD,
                                           const int32_t *sBlk, int nchunks, int stp, int wave, int lane,
                                           DCopy &dc) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int c0 = __builtin_amdgcn_readfirstlane((2 * stp + r) * NT + 64 * wave);
        const bool ok = c0 < nchunks;
        const int m = ok ? c0 >> 11 : 0;
        const int blk = __builtin_amdgcn_readfirstlane(sBlk[m]);
        const int uid = __builtin_amdgcn_readfirstlane(sBlk[64 + m]);
        const int base = 2 * (c0 & 2047);
        const double *src = du64 + (int64_t)uid * kBlockElems + base;
        dc.v[r] = *(const doublex2 *)(src + 2 * lane);
        dc.dst[r] = ok && blk >= 0 ? outD + (int64_t)blk * kBlockElems + base : nullptr;
    }
}

__device__ __forceinline__ void dcopy_store(const DCopy &dc, int lane) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (dc.dst[r]) __builtin_nontemporal_store(dc.v[r], (doublex2 *)(dc.dst[r] + 2 * lane));
}

// A class without contraction terms: between two grids, when the auxiliary
// grid is the coarser one, a stored block (J, K) can have no tile I that
// neighbours both J and K, so the sum of Eq. 15 is empty and the block is
// zero.  The workgroup clears the member tile's blocks (and gives them their
// D-hat copies), without LDS; the caller returns right after.
template <int NT, bool WD, class PD>
__device__ __forceinline__ void empty_class_tile(const PD &pd, const DevClass &cl, int m0, int rows) {
    constexpr int kChunks = kBlockElems / 2;            // 16-byte chunks of a block
    const int nm = min(rows, cl.nblocks - m0);
    for (int c = threadIdx.x; c < nm * kChunks; c += NT) {
        const int m = c / kChunks, q = c - m * kChunks;
        const int64_t blk = pd.cblk[cl.blk0 + m0 + m];
        __builtin_nontemporal_store(doublex2{0.0, 0.0}, (doublex2 *)(pd.out + blk * kBlockElems) + q);
        if constexpr (WD) {
            const int64_t u = pd.blk_uid[blk];
            __builtin_nontemporal_store(*((const doublex2 *)(pd.du64 + u * kBlockElems) + q),
                                        (doublex2 *)(pd.outD + blk * kBlockElems) + q);
        }
    }
}

// ---------------------------------------------------------------------------
// a9, FP64 MFMA class GEMM (the class decomposition is described with the
// FP32 form below).  W = N^-1 as given, M = B_IJ[p][a] B_IK[p][b] formed in
// FP64 from the transposed FP64 unique blocks.  MFMA 16x16x4 FP64: lane
// (lr, lk) holds W[16 i + lr][p] and M[p][16 j + lr] for p = 16 g + 4 lk + t;
// its result holds members 16 i + lk + 4 v of column b = 16 j + lr.  The MFMA
// accumulates in FP64 across all terms of an output row, so there is no
// separate accumulation step; four waves share a member tile and take every
// fourth row a; each step (16 pixels of one term) loads the next step's
// operands before its own MFMAs.
//
// Symmetric classes (every term pairs a unique block with itself: the blocks
// (J, J)) give C[a][b] = C[b][a] bit for bit, since the products B[p][a]
// B[p][b] are the same numbers either way round.  Row a then computes only
// the column groups j >= a / 16 (10 of the 16 16x16 tiles) and writes the
// tiles below the diagonal as mirror images (plain stores: a mirrored row
// gets its 16 values from 16 rows a at different times, and L2 merges them,
// where streaming stores would send each 8 bytes out as a partial line).
// Wave w's row x is a = w + 4 x,
// so a / 16 = x / 4: its rows run in four phases with the first column group
// JLO fixed at compile time (JLO = 0 for every row of other classes).  A step
// issues one W load per 16 members whatever the number of column groups, so
// the later phases take R rows a, a + 4, ... at once (R NI (4 - JLO) <= 16
// accumulators), sharing the W and M-column loads between them: every step
// keeps 64 MFMAs in a full tile.
// ---------------------------------------------------------------------------
template <int NI, int JLO>
struct F64Phase {
    static constexpr int NJ = 4 - JLO;
    static constexpr int R = 4 * NI * NJ <= 16 ? 4 : 2 * NI * NJ <= 16 ? 2 : 1;
    static_assert(R * NI * NJ <= 16, "a phase holds at most 16 accumulators");
};

template <int NI, bool WD>
__device__ __forceinline__ void class_f64_tile(const ProblemDesc64 &pd, int item, int32_t *sTile,
                                               int32_t *sBlk, int32_t *sTerm) {
    const double *__restrict__ ut = pd.u64t;
    const double *__restrict__ wv = pd.w;
    double *__restrict__ out = pd.out;
    const int cls = pd.mtiles[4 * item], m0 = pd.mtiles[4 * item + 1];
    const DevClass cl = pd.classes[cls];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int nterms = cl.nterms;
    const int32_t *terms = pd.cterms + 2 * cl.term0;
    if (nterms == 0) {
        empty_class_tile<256, WD>(pd, cl, m0, 16 * NI);
        return;
    }

    for (int x = threadIdx.x; x < 16 * NI * nterms; x += 256) {
        const int r = x / nterms, e = x - r * nterms;
        const int m = min(m0 + r, cl.nblocks - 1);   // rows past the class repeat its last member
        sTile[r * kTileStride + e] = pd.citab[cl.itab0 + (int64_t)m * nterms + e];
    }
    if (threadIdx.x < 64) {
        const int blk = lane < 16 * NI && m0 + lane < cl.nblocks ? pd.cblk[cl.blk0 + m0 + lane] : -1;
        sBlk[lane] = blk;
        if constexpr (WD) sBlk[64 + lane] = blk >= 0 ? pd.blk_uid[blk] : 0;   // D-hat source block
    }
    if (threadIdx.x < 2 * nterms) sTerm[threadIdx.x] = terms[threadIdx.x];   // unique-block pairs of the class
    __syncthreads();

    // operand pointers of term e for the row group starting at row a (rows
    // a + 4 r of the group lie 256 r further along u1)
    struct Ptrs { const double *w[NI], *u1, *u2; };
    auto ptrs = [&](int a, int e, Ptrs &q) {
#pragma unroll
        for (int i = 0; i < NI; ++i)
            q.w[i] = wv + (int64_t)sTile[(16 * i + lr) * kTileStride + e] * 64 + 4 * lk;
        q.u1 = ut + (int64_t)__builtin_amdgcn_readfirstlane(sTerm[2 * e]) * kBlockElems + a * 64 + 4 * lk;
        q.u2 = ut + (int64_t)__builtin_amdgcn_readfirstlane(sTerm[2 * e + 1]) * kBlockElems + lr * 64 + 4 * lk;
    };
    struct Frag { doublex4 w[NI], u1[4], u2[4]; };
    // operands of pixel group g in the shape of phase JL (its R rows, its
    // column groups >= JL)
    auto load = [&](auto jt, const Ptrs &q, int g, Frag &f) {
        constexpr int JL = decltype(jt)::value, RL = F64Phase<NI, JL>::R;
#pragma unroll
        for (int i = 0; i < NI; ++i) f.w[i] = *(const doublex4 *)(q.w[i] + 16 * g);
#pragma unroll
        for (int r = 0; r < RL; ++r) f.u1[r] = *(const doublex4 *)(q.u1 + 256 * r + 16 * g);
#pragma unroll
        for (int j = JL; j < 4; ++j) f.u2[j] = *(const doublex4 *)(q.u2 + 16 * j * 64 + 16 * g);
    };

    // accumulator of (row r of the group, member group i, column group j) in
    // phase JLO; every slot is zero between row groups
    doublex4 acc[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) acc[s] = doublex4{0.0, 0.0, 0.0, 0.0};
    constexpr int kDChunks = 16 * NI * 2048;   // D-hat chunks of the tile
    // One step of phase JLO: the loads of the next step in the shape of phase
    // JN (JLO itself, or the next phase for the last step of a phase), then
    // this step's products and MFMAs.
    auto step = [&](auto jt, auto jn, const Frag &f, const Ptrs &qn, int gn, Frag &fn, int stp, DCopy &dprev) {
        constexpr int JLO = decltype(jt)::value, NJ = F64Phase<NI, JLO>::NJ, R = F64Phase<NI, JLO>::R;
        constexpr int JN = decltype(jn)::value;
        constexpr int NLOAD = 2 * (NI + F64Phase<NI, JN>::R + F64Phase<NI, JN>::NJ);
        load(jn, qn, gn, fn);
        if constexpr (WD) {
            DCopy dc;
            dcopy_load<256>(pd.du64, pd.outD, sBlk, kDChunks, stp, wave, lane, dc);
            dcopy_store(dprev, lane);
            dprev = dc;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double bv[4][4];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = JLO; j < 4; ++j) bv[r][j] = f.u1[r][t] * f.u2[j][t];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int j = JLO; j < 4; ++j) {
                        doublex4 &c = acc[(r * NJ + j - JLO) * NI + i];
                        c = __builtin_amdgcn_mfma_f64_16x16x4f64(f.w[i][t], bv[r][j], c, 0, 0, 0);
                    }
        }
        __builtin_amdgcn_sched_group_barrier(0x020, NLOAD, 0);          // loads first
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            __builtin_amdgcn_sched_group_barrier(0x002, R * NJ, 0);      // products of pixel t
            __builtin_amdgcn_sched_group_barrier(0x008, R * NJ * NI, 0); // their MFMAs
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    // end of a row group (first row x): store groups >= JLO of its rows (and
    // their mirror images below the diagonal in a symmetric class), clear
    auto store_group = [&](auto jt, auto symt, int x) {
        constexpr int JLO = decltype(jt)::value, NJ = F64Phase<NI, JLO>::NJ, R = F64Phase<NI, JLO>::R;
        constexpr bool SYM = decltype(symt)::value;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int a = wave + 4 * (x + r);
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int blk = sBlk[16 * i + lk + 4 * v];
                    if (blk >= 0) {
                        double *ob = out + (int64_t)blk * kBlockElems;
#pragma unroll
                        for (int j = JLO; j < 4; ++j)
                            __builtin_nontemporal_store(acc[(r * NJ + j - JLO) * NI + i][v], &ob[a * 64 + 16 * j + lr]);
                        if constexpr (SYM) {
#pragma unroll
                            for (int j = JLO + 1; j < 4; ++j)
                                ob[(16 * j + lr) * 64 + a] = acc[(r * NJ + j - JLO) * NI + i][v];
                        }
                    }
                }
        }
#pragma unroll
        for (int s = 0; s < R * NJ * NI; ++s) acc[s] = doublex4{0.0, 0.0, 0.0, 0.0};
    };

    Frag f0, f1;
    Ptrs qc, qn;
    int it = 0;                          // (row group, term) iterations done: 4 steps each
    DCopy dpend;                         // D-hat chunks loaded, not yet stored
    dpend.dst[0] = dpend.dst[1] = nullptr;
    // rows x in [xb, xe) of phase JLO in groups of R; JN: the phase after it.
    // One (row group x, term e) iteration is four steps; the last iteration of
    // the phase is peeled, so that the operands it loads in the next phase's
    // shape are live only from there on.
    auto phase = [&](auto jt, auto jn, auto symt, int xb, int xe) {
        constexpr int R = F64Phase<NI, decltype(jt)::value>::R;
        auto iteration = [&](auto jl, int x, int e) {
            const bool last_term = e + 1 == nterms;
            const int nx = last_term ? x + R : x, ne = last_term ? 0 : e + 1;
            if (nx < 16) ptrs(wave + 4 * nx, ne, qn);
            else qn = qc;                // past the last row: a harmless reload
            step(jt, jt, f0, qc, 1, f1, 4 * it, dpend);
            step(jt, jt, f1, qc, 2, f0, 4 * it + 1, dpend);
            step(jt, jt, f0, qc, 3, f1, 4 * it + 2, dpend);
            step(jt, jl, f1, qn, 0, f0, 4 * it + 3, dpend);
            if (last_term) store_group(jt, symt, x);
            qc = qn;
            ++it;
        };
        const int n_iter = (xe - xb) / R * nterms;
        int x = xb, e = 0;
        for (int n = 0; n + 1 < n_iter; ++n) {
            iteration(jt, x, e);
            if (++e == nterms) {
                e = 0;
                x += R;
            }
        }
        iteration(jn, x, e);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    ptrs(wave, 0, qc);
    load(I0(), qc, 0, f0);
    if (cl.sym != 0) {
        phase(I0(), I1(), std::true_type(), 0, 4);
        phase(I1(), I2(), std::true_type(), 4, 8);
        phase(I2(), I3(), std::true_type(), 8, 12);
        phase(I3(), I3(), std::true_type(), 12, 16);
    } else {
        phase(I0(), I0(), std::false_type(), 0, 16);
    }
    if constexpr (WD) {                  // the last step's chunks, then those past the last step
        dcopy_store(dpend, lane);
        for (int stp = 4 * it; 512 * stp < kDChunks; ++stp) {
            DCopy dc;
            dcopy_load<256>(pd.du64, pd.outD, sBlk, kDChunks, stp, wave, lane, dc);
            dcopy_store(dc, lane);
        }
    }
}

template <bool WD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_class_f64(ProblemDesc64 pd) {
    __shared__ int32_t sTile[64 * kTileStride];
    __shared__ int32_t sBlk[128];                    // stored block per member row; D-hat source block
    __shared__ int32_t sTerm[2 * kMaxClassTerms];     // unique-block pairs of the class
    const int item = blockIdx.x;        // pd.mtiles: a dispatch table, slot per workgroup
    const int groups = pd.mtiles[4 * item + 2];
    if (groups == 0) return;            // an empty slot
    if (groups == 4) class_f64_tile<4, WD>(pd, item, sTile, sBlk, sTerm);
    else if (groups == 2) class_f64_tile<2, WD>(pd, item, sTile, sBlk, sTerm);
    else class_f64_tile<1, WD>(pd, item, sTile, sBlk, sTerm);
}

// Queue draining shared by the persistent batch kernels: thread 0 takes the
// next item from queue home, then steals from the others in order; -1 once
// every queue is empty.  Counters only grow, so every workgroup leaves.
__device__ __forceinline__ int batch_next_item(const int32_t *__restrict__ qb, int32_t nq,
                                               int32_t *__restrict__ counters, int home, int &tried) {
    int it = -1;
    while (tried < nq) {
        const int q = (home + tried) % nq;
        const int c = atomicAdd(&counters[q], 1);
        if (c < qb[q + 1] - qb[q]) {
            it = qb[q] + c;
            break;
        }
        ++tried;
    }
    return it;
}

// a10 in FP64: the FP64 class GEMM of many problems in one persistent launch
// (one 4-wave workgroup per CU, as k_class_f64), fed by the same queues as the
// FP32 and split-BF16 batch kernels below.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_batch_f64(const ProblemDesc64 *__restrict__ probs, const int32_t *__restrict__ items,
                 const int32_t *__restrict__ qb, int32_t nq, int32_t *__restrict__ counters) {
    __shared__ int32_t sTile[64 * kTileStride];
    __shared__ int32_t sBlk[128];
    __shared__ int32_t sTerm[2 * kMaxClassTerms];
    __shared__ int32_t sItem;
    const int home = blockIdx.x % nq;
    int tried = 0;                       // queues found empty (thread 0)
    for (;;) {
        if (threadIdx.x == 0) sItem = batch_next_item(qb, nq, counters, home, tried);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(sItem);   // uniform: descriptors in scalar registers
        __syncthreads();                 // every thread has read sItem before it changes
        if (it < 0) break;
        const ProblemDesc64 pd = probs[items[2 * it]];
        const int item = items[2 * it + 1];
        const int groups = pd.mtiles[4 * item + 2];
        if (groups == 4) class_f64_tile<4, false>(pd, item, sTile, sBlk, sTerm);
        else if (groups == 2) class_f64_tile<2, false>(pd, item, sTile, sBlk, sTerm);
        else class_f64_tile<1, false>(pd, item, sTile, sBlk, sTerm);
    }
}

// ---------------------------------------------------------------------------
// a9, FP32 MFMA class GEMM.  Same decomposition as the split-BF16 form below:
// C[m][(a,b)] = sum_(e,p) W[m][(e,p)] M[(e,p)][(a,b)], W = N^-1 rounded to FP32,
// M = B_IJ[p][a] B_IK[p][b] formed as the FP32 product of the FP32 copies.
// The same schedule as the split-BF16 kernel: eight waves per member tile,
// wave w the output rows a = w mod 4 and the column half w / 4, two waves per
// SIMD; W and the B_IK values of a step (32 pixels) staged through four LDS
// buffers two steps ahead, one barrier per term.  MFMA 16x16x4 FP32, MFMA g
// of a step taking the pixels 8 lk + g; the result lane holds members
// 16 i + 4 lk + v of column b = 16 j + lr.  A term's FP32 sum over its 64
// pixels is added to FP64 accumulators, which are stored and cleared at the
// end of every row a.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ninv_f32(const double *__restrict__ ninv, int64_t n,
                                                  float *__restrict__ wf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wf[i] = (float)ninv[i];
}

// One member tile (item) of one problem with NI groups of 16 member rows; all
// 512 threads of the workgroup take part.  sTile / sBlk / sTerm are the
// workgroup's LDS tables, sW / sU its four staging buffers.
template <int NI, bool WD>
__device__ __forceinline__ void class_f32_tile(const ProblemDesc &pd, int item, int32_t *sTile,
                                               int32_t *sBlk, int32_t *sTerm, floatx4 *sW, floatx4 *sU) {
    const float *__restrict__ ut32 = pd.ut32;
    double *__restrict__ out = pd.out;
    constexpr int NW = 8, NT = 64 * NW, RP = NW / 2, RPW = 64 / RP;
    const int cls = pd.mtiles[4 * item], m0 = pd.mtiles[4 * item + 1];
    const DevClass cl = pd.classes[cls];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rw = wave % RP, ch = wave / RP;          // row phase, column half
    const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int nterms = cl.nterms;
    const int32_t *terms = pd.cterms + 2 * cl.term0;
    if (nterms == 0) {
        empty_class_tile<NT, WD>(pd, cl, m0, 16 * NI);
        return;
    }

    for (int x = tid; x < 16 * NI * nterms; x += NT) {
        const int r = x / nterms, e = x - r * nterms;
        const int m = min(m0 + r, cl.nblocks - 1);   // rows past the class repeat its last member
        sTile[r * kTileStride + e] = pd.citab[cl.itab0 + (int64_t)m * nterms + e];
    }
    if (tid < 64) {
        const int blk = lane < 16 * NI && m0 + lane < cl.nblocks ? pd.cblk[cl.blk0 + m0 + lane] : -1;
        sBlk[lane] = blk;
        if constexpr (WD) sBlk[64 + lane] = blk >= 0 ? pd.blk_uid[blk] : 0;   // D-hat source block
    }
    if (tid < 2 * nterms) sTerm[tid] = terms[tid];   // unique-block pairs of the class
    __syncthreads();

    // Staging of one step (32 pixels of a term): W of the tile's 64 rows and
    // the B_IK values of its 64 columns, FP32, 8 chunks of 16 bytes per row
    // each; thread t takes W chunk t (row t >> 3) and B_IK chunk t.  Rows past
    // the tile's 16 NI members load the last member's values into LDS rows no
    // wave reads.  LDS row r keeps its chunk c at 8 r + (c ^ usw(r)).
    auto usw = [](int b) { return ((b >> 1) ^ (b << 2)) & 7; };
    const int srow = tid >> 3, sch = tid & 7;
    const int wrow = min(srow, 16 * NI - 1) * kTileStride;
    const int sdst = srow * 8 + (sch ^ usw(srow));
    struct SAddr { int64_t wo; const float *u2; };
    struct OAddr { const float *p1; };
    auto saddr = [&](int e, int h) {
        SAddr r;
        r.wo = (int64_t)sTile[wrow + e] * 64 + 32 * h + 4 * sch;
        r.u2 = ut32 + (int64_t)__builtin_amdgcn_readfirstlane(sTerm[2 * e + 1]) * kBlockElems + 32 * h;
        return r;
    };
    // this lane's B_IJ values of row a: pixels 32 h + 8 lk + g, g = 0..7
    auto oaddr = [&](int a, int e, int h) {
        OAddr r;
        r.p1 = ut32 + (int64_t)__builtin_amdgcn_readfirstlane(sTerm[2 * e]) * kBlockElems + a * 64 + 32 * h + 8 * lk;
        return r;
    };
    struct Stage { floatx4 w, u; };
    struct Own { floatx4 u1[2]; };
    auto stage_load = [&](const SAddr &ad, Stage &st) {
        st.w = *(const floatx4 *)(pd.wf + ad.wo);
        st.u = *(const floatx4 *)(ad.u2 + srow * 64 + 4 * sch);
    };
    auto own_load = [&](const OAddr &ad, Own &o) {
        o.u1[0] = *(const floatx4 *)ad.p1;
        o.u1[1] = *(const floatx4 *)(ad.p1 + 4);
    };
    auto stage_store = [&](const Stage &st, int buf) {
        sW[buf * 512 + sdst] = st.w;
        sU[buf * 512 + sdst] = st.u;
    };
    constexpr int kDChunks = 16 * NI * 2048;   // D-hat chunks of the tile

    doublex4 acc[NI][2];
    floatx4 part[NI][2];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    // One step, in three scheduling regions as in the split-BF16 form.  MFMA
    // g (g = 0..7) of a step takes the pixels 8 lk + g: lane (lr, lk) holds
    // W[16 i + lr][8 lk + g] and M[8 lk + g][16 j + lr].
    auto step = [&](const Own &oc, int buf, const SAddr &sa, const OAddr &oa, int sbuf, Stage &stn, Own &on,
                    bool first, bool bar, int nse, int nsh, int noa, int noe, int noh, SAddr &sa_n, OAddr &oa_n,
                    int stp, DCopy &dprev, auto symt, int ng, int g0, int g1) {
        constexpr bool S = decltype(symt)::value;
        stage_load(sa, stn);
        own_load(oa, on);
        if constexpr (WD) {
            DCopy dc;
            dcopy_load<NT>(pd.du64, pd.outD, sBlk, kDChunks, stp, wave, lane, dc);
            dcopy_store(dprev, lane);
            dprev = dc;
        }
        __builtin_amdgcn_sched_barrier(0);
        floatx4 wfr[NI][2];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int r = 16 * i + lr;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) wfr[i][hh] = sW[buf * 512 + r * 8 + ((2 * lk + hh) ^ usw(r))];
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            if (S && jj >= ng) continue;     // symmetric class: this wave's groups of the row
            const int b = S ? 16 * (jj ? g1 : g0) + lr : 32 * ch + 16 * jj + lr;
            float m[8];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const floatx4 u2 = sU[buf * 512 + b * 8 + ((2 * lk + hh) ^ usw(b))];
#pragma unroll
                for (int t = 0; t < 4; ++t) m[4 * hh + t] = oc.u1[hh][t] * u2[t];
            }
#pragma unroll
            for (int g = 0; g < 8; ++g)
#pragma unroll
                for (int i = 0; i < NI; ++i)
                    part[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        wfr[i][g >> 2][g & 3], m[g], (first && g == 0) ? floatx4{0.f, 0.f, 0.f, 0.f} : part[i][jj], 0, 0, 0);
        }
        sa_n = saddr(nse, nsh);
        oa_n = oaddr(noa, noe, noh);
        __builtin_amdgcn_sched_barrier(0);
        stage_store(stn, sbuf);
        if (bar) __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
    };

    // Four LDS buffers: iteration it (one term of one row) computes from
    // buffers 2 (it & 1) + h, fills the other pair for iteration it + 1, and
    // ends with the only barrier of the term.
    auto next = [&](int cx, int ce, int &nx, int &ne) {
        ne = ce + 1;
        nx = cx;
        if (ne == nterms) {
            ne = 0;
            ++nx;
        }
        if (nx >= RPW) {
            nx = cx;
            ne = ce;
        }
    };
    Stage s0, s1;
    Own o0, o1;
    int x = 0, e = 0;
    int x1, e1;
    next(0, 0, x1, e1);
    {
        Stage t0, t1;
        stage_load(saddr(0, 0), t0);
        stage_load(saddr(0, 1), t1);
        own_load(oaddr(rw, 0, 0), o0);
        stage_store(t0, 0);
        stage_store(t1, 1);
    }
    SAddr sa = saddr(e1, 0);
    OAddr oa = oaddr(rw, 0, 1);
    DCopy dpend;                           // D-hat chunks loaded, not yet stored
    dpend.dst[0] = dpend.dst[1] = nullptr;
    __syncthreads();
    // Symmetric classes (every term pairs a unique block with itself: the
    // blocks (J, J), with C[a][b] = C[b][a] bit for bit since the products
    // B[p][a] B[p][b] are the same numbers either way round): row a needs only
    // the column groups j >= a / 16 (= x / 4, as a = rw + 4 x); the tiles
    // below the diagonal are written as mirror images.  The groups a row needs
    // are shared out so that the two waves of a row phase (column halves 0
    // and 1) do at most two groups each and one each where two are left:
    // x / 4 = 0: {0, 1} | {2, 3};  1: {1} | {2, 3};  2: {2} | {3};  3: {} | {3}.
    auto rows = [&](auto symt) {
        constexpr bool S = decltype(symt)::value;
        for (int it = 0; it < RPW * nterms; ++it) {
            next(x, e, x1, e1);
            const int a = rw + RP * x, a1 = rw + RP * x1;
            int x2, e2;
            next(x1, e1, x2, e2);
            const int p = x >> 2;
            int ng = 2, g0 = 2 * ch, g1 = 2 * ch + 1;
            if constexpr (S) {
                if (p == 1 && ch == 0) {
                    ng = 1;
                    g0 = 1;
                } else if (p == 2) {
                    ng = 1;
                    g0 = 2 + ch;
                } else if (p == 3) {
                    ng = ch;
                    g0 = 3;
                }
            }
            const int ib = 2 * (it & 1), nb = 2 - ib;
            step(o0, ib, sa, oa, nb, s1, o1, true, false, e1, 1, a1, e1, 0, sa, oa, 2 * it, dpend, symt, ng, g0, g1);
            step(o1, ib + 1, sa, oa, nb + 1, s0, o0, false, true, e2, 0, a1, e1, 1, sa, oa, 2 * it + 1, dpend, symt,
                 ng, g0, g1);
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (!S || j < ng) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)part[i][j][v];
                    }
            if (e == nterms - 1) {           // end of output row a: store, clear
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int blk = sBlk[16 * i + 4 * lk + v];
                        if (blk >= 0) {
                            double *ob = out + (int64_t)blk * kBlockElems;
#pragma unroll
                            for (int j = 0; j < 2; ++j) {
                                if (S && j >= ng) continue;
                                const int G = S ? (j ? g1 : g0) : 2 * ch + j;
                                __builtin_nontemporal_store(acc[i][j][v], &ob[a * 64 + 16 * G + lr]);
                                if (S && G > p) ob[(16 * G + lr) * 64 + a] = acc[i][j][v];
                            }
                        }
                    }
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
            }
            x = x1;
            e = e1;
        }
    };
    if (cl.sym != 0) rows(std::true_type());
    else rows(std::false_type());
    if constexpr (WD) {                  // the last step's chunks, then those past the last step
        dcopy_store(dpend, lane);
        for (int stp = 2 * RPW * nterms; 2 * NT * stp < kDChunks; ++stp) {
            DCopy dc;
            dcopy_load<NT>(pd.du64, pd.outD, sBlk, kDChunks, stp, wave, lane, dc);
            dcopy_store(dc, lane);
        }
    }
}

template <bool WD>
__device__ __forceinline__ void class_f32_item(const ProblemDesc &pd, int item, int32_t *sTile, int32_t *sBlk,
                                               int32_t *sTerm, floatx4 *sW, floatx4 *sU) {
    const int groups = pd.mtiles[4 * item + 2];
    if (groups == 0) return;            // an empty slot of a dispatch table
    if (groups == 4) class_f32_tile<4, WD>(pd, item, sTile, sBlk, sTerm, sW, sU);
    else if (groups == 2) class_f32_tile<2, WD>(pd, item, sTile, sBlk, sTerm, sW, sU);
    else class_f32_tile<1, WD>(pd, item, sTile, sBlk, sTerm, sW, sU);
}

template <bool WD>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_class_f32(ProblemDesc pd) {
    __shared__ int32_t sTile[64 * kTileStride];   // tile I of (member row, term)
    __shared__ int32_t sBlk[128];                    // stored block per member row; D-hat source block
    __shared__ int32_t sTerm[2 * kMaxClassTerms];     // unique-block pairs of the class
    __shared__ floatx4 sW[4 * 512];                  // staged W, four buffers
    __shared__ floatx4 sU[4 * 512];                  // staged B_IK values, four buffers
    class_f32_item<WD>(pd, blockIdx.x, sTile, sBlk, sTerm, sW, sU);
}

// ---------------------------------------------------------------------------
// a10: many problems in one persistent launch.  Work items (problem, member
// tile) sit in nq queues, queue q holding items [qb[q], qb[q+1]).  Workgroup b
// drains queue b mod nq first (with one queue per XCD and items in natural
// order, the tiles an XCD runs together share operands in its L2), then steals
// from the others.  Counters only grow, so every workgroup leaves once all
// queues are empty.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_fill_i32(int32_t *p, int32_t n, int32_t v) {
    for (int i = threadIdx.x; i < n; i += 64) p[i] = v;
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_batch_f32(const ProblemDesc *__restrict__ probs, const int32_t *__restrict__ items,
                 const int32_t *__restrict__ qb, int32_t nq, int32_t *__restrict__ counters) {
    __shared__ int32_t sTile[64 * kTileStride];
    __shared__ int32_t sBlk[128];
    __shared__ int32_t sTerm[2 * kMaxClassTerms];     // unique-block pairs of the class
    __shared__ floatx4 sW[4 * 512];
    __shared__ floatx4 sU[4 * 512];
    __shared__ int32_t sItem;
    const int home = blockIdx.x % nq;
    int tried = 0;                       // queues found empty (thread 0)
    for (;;) {
        if (threadIdx.x == 0) sItem = batch_next_item(qb, nq, counters, home, tried);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(sItem);   // uniform: descriptors in scalar registers
        __syncthreads();                 // every thread has read sItem before it changes
        if (it < 0) break;
        const ProblemDesc pd = probs[items[2 * it]];
        class_f32_item<false>(pd, items[2 * it + 1], sTile, sBlk, sTerm, sW, sU);
    }
}

// ---------------------------------------------------------------------------
// a9, split BF16.  A value is split into NP BF16 parts, each rounded to nearest
// even from the exact FP32 remainder of the previous ones: three parts
// represent an FP32 value exactly, two parts to 2^-17 relative, and every
// part has a sign independent of the value's, so the products left out
// (NP = 3: ml, lm, ll; NP = 2: mm) are unbiased.  Products kept: NP = 3: mm,
// lh, hl, mh, hm, hh (all of order >= 2^-16); NP = 2: mh, hm, hh.  FP32 MFMA
// accumulation over the 64 pixels of one contraction tile, FP64 across tiles.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {   // round to nearest even
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){a, b}, bf16x2));
}

template <int NP>
__device__ __forceinline__ void split_pair(float y0, float y1, uint32_t *out) {
    const uint32_t h = pack_bf16(y0, y1);
    out[0] = h;
    const float r0 = y0 - __uint_as_float(h << 16);
    const float r1 = y1 - __uint_as_float(h & 0xffff0000u);
    const uint32_t m = pack_bf16(r0, r1);
    out[1] = m;
    if constexpr (NP == 3) {
        const float l0 = r0 - __uint_as_float(m << 16);
        const float l1 = r1 - __uint_as_float(m & 0xffff0000u);
        out[2] = pack_bf16(l0, l1);
    }
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *(const u16x8 *)p);
}

// N^-1 split into three BF16 parts (hi, mid, lo) from FP64, read directly as
// MFMA operands by the class GEMM.
__global__ __launch_bounds__(256) void k_split_ninv(const double *__restrict__ ninv, int64_t n,
                                                    uint16_t *__restrict__ w0, uint16_t *__restrict__ w1,
                                                    uint16_t *__restrict__ w2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = ninv[i];
    const uint16_t h = bf16_bits((float)v);
    const double r1 = v - (double)bf16_value(h);
    const uint16_t m = bf16_bits((float)r1);
    w0[i] = h;
    w1[i] = m;
    w2[i] = bf16_bits((float)(r1 - (double)bf16_value(m)));
}

// Split-BF16 class GEMM (the decomposition of the FP32 form above): W = N^-1
// split into NP BF16 parts, M = B_IJ[p][a] B_IK[p][b] formed as an FP32
// product and split into NP parts in registers; NP = 3 keeps the products hh,
// hm, mh, hl, lh, mm (smallest first), NP = 2 keeps hh, hm, mh.  MFMA
// 16x16x32 BF16: lane (lr, lk) holds W[16 i + lr][p0 + 8 lk + 0..7] and
// M[p0 + 8 lk + 0..7][16 j + lr]; the result holds members 16 i + 4 lk + v.
// Eight waves per member tile, two on each SIMD: a wave's own VALU work
// (forming and splitting M, the FP64 accumulation) does not overlap its
// MFMAs, but it does overlap those of the other wave on its SIMD.  Wave w
// takes the output rows a = w mod 4 and the column half w / 4, so each wave
// holds half the columns of its rows.  The operands all waves share (W of the tile's
// rows, the B_IK values of a step) are staged through LDS.  A step is 32
// pixels (half a term); a term's FP32 sums are added to the FP64 accumulators
// after its second step.
// With WD the launch also writes D-hat: the D-hat block of every stored block
// of the tile is its unique block, copied in 16-byte chunks, two per thread
// and step (loaded with one step's loads, stored after the next step's), so
// that these writes proceed under the contraction's arithmetic; chunks left
// after the last step are copied at the end of the tile.
template <int NP, int NI, bool WD>
__device__ __forceinline__ void class_bf16_tile(const ProblemDescB &pd, int item, int32_t *sTile,
                                                int32_t *sBlk, int32_t *sTerm, u16x8 *sW, floatx4 *sU) {
    const float *__restrict__ ut32 = pd.ut32;
    double *__restrict__ out = pd.out;
    const int cls = pd.mtiles[4 * item], m0 = pd.mtiles[4 * item + 1];
    const DevClass cl = pd.classes[cls];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int NW = 8, NT = 64 * NW;              // waves, threads
    constexpr int RP = NW / 2, RPW = 64 / RP;          // row phases, rows per wave
    const int rw = wave % RP, ch = wave / RP;          // row phase, column half
    const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int nterms = cl.nterms;
    const int32_t *terms = pd.cterms + 2 * cl.term0;
    if (nterms == 0) {
        empty_class_tile<NT, WD>(pd, cl, m0, 16 * NI);
        return;
    }

    for (int x = tid; x < 16 * NI * nterms; x += NT) {
        const int r = x / nterms, e = x - r * nterms;
        const int m = min(m0 + r, cl.nblocks - 1);   // rows past the class repeat its last member
        sTile[r * kTileStride + e] = pd.citab[cl.itab0 + (int64_t)m * nterms + e];
    }
    if (tid < 64) {
        const int blk = lane < 16 * NI && m0 + lane < cl.nblocks ? pd.cblk[cl.blk0 + m0 + lane] : -1;
        sBlk[lane] = blk;
        if constexpr (WD) sBlk[64 + lane] = blk >= 0 ? pd.blk_uid[blk] : 0;   // D-hat source block
    }
    if (tid < 2 * nterms) sTerm[tid] = terms[tid];   // unique-block pairs of the class
    __syncthreads();

    // Staging: W is 256 NP chunks of 16 bytes (part c >> 8, row (c & 255) >> 2,
    // chunk c & 3), B_IK of one step 512 chunks (row c >> 3, chunk c & 7).
    // Thread t takes W chunks t + NT r and B_IK chunks t + NT q; with 512
    // threads and NP = 3 the threads past the last W chunk repeat one (same
    // value to the same LDS place), so every thread issues the same loads.
    // Rows past the tile's 16 NI members load the last member's values into
    // LDS rows no wave reads.
    constexpr int NWC = (256 * NP + NT - 1) / NT, NUC = 512 / NT;
    const uint16_t *wsrc[NWC];
    int wrow[NWC], wdst[NWC];
    auto wsw = [](int r) { return ((r >> 1) ^ (r >> 3)) & 3; };
    auto usw = [](int b) { return ((b >> 1) ^ (b << 2)) & 7; };
#pragma unroll
    for (int r = 0; r < NWC; ++r) {
        int c = tid + NT * r;
        if (c >= 256 * NP) c -= 256;
        const int k = __builtin_amdgcn_readfirstlane(c >> 8), q = c & 255, row = q >> 2, sub = q & 3;
        wsrc[r] = pd.w[k] + 8 * sub;
        wrow[r] = min(row, 16 * NI - 1) * kTileStride;
        // LDS layouts, in 16-byte chunks: W row r (64 bytes) keeps its chunk c at
        // 4 r + (c ^ wsw(r)), a B_IK row b (128 bytes) its chunk c at 8 b + (c ^
        // usw(b)); every read and write phase then touches distinct banks,
        // whether a 16-byte access is served 8 lanes at a time over 32 banks or
        // 16 lanes at a time over 64 banks.
        wdst[r] = (k * 64 + row) * 4 + (sub ^ wsw(row));
    }
    int usrc[NUC], udst[NUC];
#pragma unroll
    for (int q = 0; q < NUC; ++q) {
        const int c = tid + NT * q, ub = c >> 3, uc = c & 7;
        usrc[q] = ub * 64 + 4 * uc;
        udst[q] = ub * 8 + (uc ^ usw(ub));
    }

    // Addresses of one step (term e, half h) for the staged operands (W
    // offsets of this thread's chunks, B_IK rows), and of this lane's B_IJ
    // values of row a.
    struct SAddr { int64_t wo[NWC]; const float *u2; };
    struct OAddr { const float *p1; };
    auto saddr = [&](int e, int h) {
        SAddr r;
#pragma unroll
        for (int q = 0; q < NWC; ++q) r.wo[q] = (int64_t)sTile[wrow[q] + e] * 64 + 32 * h;
        r.u2 = ut32 + (int64_t)__builtin_amdgcn_readfirstlane(sTerm[2 * e + 1]) * kBlockElems + 32 * h;
        return r;
    };
    auto oaddr = [&](int a, int e, int h) {
        OAddr r;
        r.p1 = ut32 + (int64_t)__builtin_amdgcn_readfirstlane(sTerm[2 * e]) * kBlockElems + a * 64 + 32 * h + 8 * lk;
        return r;
    };
    struct Stage { u16x8 w[NWC]; floatx4 u[NUC]; };
    struct Own { floatx4 u1[2]; };        // B_IJ values of this wave's output row (not shared)
    auto stage_load = [&](const SAddr &ad, Stage &st) {
#pragma unroll
        for (int q = 0; q < NWC; ++q) st.w[q] = *(const u16x8 *)(wsrc[q] + ad.wo[q]);
#pragma unroll
        for (int q = 0; q < NUC; ++q) st.u[q] = *(const floatx4 *)(ad.u2 + usrc[q]);
    };
    auto own_load = [&](const OAddr &ad, Own &o) {
        o.u1[0] = *(const floatx4 *)ad.p1;
        o.u1[1] = *(const floatx4 *)(ad.p1 + 4);
    };
    auto stage_store = [&](const Stage &st, int buf) {
#pragma unroll
        for (int q = 0; q < NWC; ++q) sW[buf * NP * 256 + wdst[q]] = st.w[q];
#pragma unroll
        for (int q = 0; q < NUC; ++q) sU[buf * 512 + udst[q]] = st.u[q];
    };
    constexpr int kDChunks = 16 * NI * 2048;   // D-hat chunks of the tile

    doublex4 acc[NI][2];
    floatx4 part[NI][2];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    constexpr int NPROD = NP == 3 ? 6 : 3;
    // One step, in three scheduling regions: (1) the loads of the staged
    // operands of the step two ahead and of this wave's B_IJ values of the
    // next step; (2) the MFMAs of this step from LDS buffer buf (W fragments,
    // and M formed from the staged B_IK values and this wave's B_IJ values),
    // with the addresses the next step needs read meanwhile; (3) the staged
    // operands written to buffer sbuf, and, at the end of a term, a barrier.
    auto step = [&](const Own &oc, int buf, const SAddr &sa, const OAddr &oa, int sbuf, Stage &stn, Own &on,
                    bool first, bool bar, int nse, int nsh, int noa, int noe, int noh, SAddr &sa_n, OAddr &oa_n,
                    int stp, DCopy &dprev, auto symt, int ng, int g0, int g1) {
        constexpr bool S = decltype(symt)::value;
        stage_load(sa, stn);
        own_load(oa, on);
        if constexpr (WD) {
            DCopy dc;
            dcopy_load<NT>(pd.du64, pd.outD, sBlk, kDChunks, stp, wave, lane, dc);
            dcopy_store(dprev, lane);
            dprev = dc;
        }
        __builtin_amdgcn_sched_barrier(0);
        bf16x8 wf[NI][NP];
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int k = 0; k < NP; ++k)
                wf[i][k] = __builtin_bit_cast(bf16x8, sW[((buf * NP + k) * 64 + 16 * i + lr) * 4 + (lk ^ wsw(16 * i + lr))]);
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            if (S && jj >= ng) continue;     // symmetric class: this wave's groups of the row
            const int b = S ? 16 * (jj ? g1 : g0) + lr : 32 * ch + 16 * jj + lr;
            const floatx4 u2a = sU[buf * 512 + b * 8 + ((2 * lk) ^ usw(b))];
            const floatx4 u2b = sU[buf * 512 + b * 8 + ((2 * lk + 1) ^ usw(b))];
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            u32x4 words[NP];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int hh = q >> 1, y = 2 * (q & 1);
                const floatx4 &u2 = hh ? u2b : u2a;
                uint32_t parts[NP];
                split_pair<NP>(oc.u1[hh][y] * u2[y], oc.u1[hh][y + 1] * u2[y + 1], parts);
#pragma unroll
                for (int k = 0; k < NP; ++k) words[k][q] = parts[k];
            }
            bf16x8 bfr[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) bfr[k] = __builtin_bit_cast(bf16x8, words[k]);
            constexpr int pa3[6] = {1, 2, 0, 1, 0, 0}, pb3[6] = {1, 0, 2, 0, 1, 0};
            constexpr int pa2[3] = {1, 0, 0}, pb2[3] = {0, 1, 0};
#pragma unroll
            for (int pr = 0; pr < NPROD; ++pr) {
                const int qa = NP == 3 ? pa3[pr] : pa2[pr];
                const int qb = NP == 3 ? pb3[pr] : pb2[pr];
#pragma unroll
                for (int i = 0; i < NI; ++i)
                    part[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        wf[i][qa], bfr[qb], (first && pr == 0) ? floatx4{0.f, 0.f, 0.f, 0.f} : part[i][jj], 0, 0, 0);
            }
        }
        sa_n = saddr(nse, nsh);
        oa_n = oaddr(noa, noe, noh);
        __builtin_amdgcn_sched_group_barrier(0x100, NI * NP + 6 + NWC, 0);   // LDS reads
#pragma unroll
        for (int x = 0; x < 2 * NPROD * NI; ++x) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);             // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);             // two VALU
        }
        __builtin_amdgcn_sched_barrier(0);
        stage_store(stn, sbuf);
        if (bar) __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
    };

    // Four LDS buffers: iteration it (one term of one row) computes from
    // buffers 2 (it & 1) + h, fills the other pair for iteration it + 1, and
    // ends with the only barrier of the term.  Cursors: row index x
    // (a = rw + RP x) and term e; past the last row they repeat (harmless
    // reloads into buffers no step reads).
    auto next = [&](int cx, int ce, int &nx, int &ne) {
        ne = ce + 1;
        nx = cx;
        if (ne == nterms) {
            ne = 0;
            ++nx;
        }
        if (nx >= RPW) {
            nx = cx;
            ne = ce;
        }
    };
    Stage s0, s1;
    Own o0, o1;
    int x = 0, e = 0;
    int x1, e1;
    next(0, 0, x1, e1);
    {
        Stage t0, t1;
        stage_load(saddr(0, 0), t0);
        stage_load(saddr(0, 1), t1);
        own_load(oaddr(rw, 0, 0), o0);
        stage_store(t0, 0);
        stage_store(t1, 1);
    }
    SAddr sa = saddr(e1, 0);
    OAddr oa = oaddr(rw, 0, 1);
    DCopy dpend;                           // D-hat chunks loaded, not yet stored
    dpend.dst[0] = dpend.dst[1] = nullptr;
    __syncthreads();
    // Symmetric classes (every term pairs a unique block with itself: the
    // blocks (J, J), with C[a][b] = C[b][a] bit for bit since the products
    // B[p][a] B[p][b] are the same numbers either way round): row a needs only
    // the column groups j >= a / 16 (= x / 4, as a = rw + 4 x); the tiles
    // below the diagonal are written as mirror images.  The groups a row needs
    // are shared out so that the two waves of a row phase (column halves 0
    // and 1) do at most two groups each and one each where two are left:
    // x / 4 = 0: {0, 1} | {2, 3};  1: {1} | {2, 3};  2: {2} | {3};  3: {} | {3}.
    auto rows = [&](auto symt) {
        constexpr bool S = decltype(symt)::value;
        for (int it = 0; it < RPW * nterms; ++it) {
            next(x, e, x1, e1);
            const int a = rw + RP * x, a1 = rw + RP * x1;
            int x2, e2;
            next(x1, e1, x2, e2);
            const int p = x >> 2;
            int ng = 2, g0 = 2 * ch, g1 = 2 * ch + 1;
            if constexpr (S) {
                if (p == 1 && ch == 0) {
                    ng = 1;
                    g0 = 1;
                } else if (p == 2) {
                    ng = 1;
                    g0 = 2 + ch;
                } else if (p == 3) {
                    ng = ch;
                    g0 = 3;
                }
            }
            const int ib = 2 * (it & 1), nb = 2 - ib;
            step(o0, ib, sa, oa, nb, s1, o1, true, false, e1, 1, a1, e1, 0, sa, oa, 2 * it, dpend, symt, ng, g0, g1);
            step(o1, ib + 1, sa, oa, nb + 1, s0, o0, false, true, e2, 0, a1, e1, 1, sa, oa, 2 * it + 1, dpend, symt,
                 ng, g0, g1);
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (!S || j < ng) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)part[i][j][v];
                    }
            if (e == nterms - 1) {           // end of output row a: store, clear
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int blk = sBlk[16 * i + 4 * lk + v];
                        if (blk >= 0) {
                            double *ob = out + (int64_t)blk * kBlockElems;
#pragma unroll
                            for (int j = 0; j < 2; ++j) {
                                if (S && j >= ng) continue;
                                const int G = S ? (j ? g1 : g0) : 2 * ch + j;
                                __builtin_nontemporal_store(acc[i][j][v], &ob[a * 64 + 16 * G + lr]);
                                if (S && G > p) ob[(16 * G + lr) * 64 + a] = acc[i][j][v];
                            }
                        }
                    }
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
            }
            x = x1;
            e = e1;
        }
    };
    // The symmetric sharing of column groups is not used here: its branches
    // inside the step cost the split-BF16 form more (the step's scheduling
    // regions, code size) than the skipped groups save (measured).
    rows(std::false_type());
    if constexpr (WD) {                  // the last step's chunks, then those past the last step
        dcopy_store(dpend, lane);
        for (int stp = 2 * RPW * nterms; 2 * NT * stp < kDChunks; ++stp) {
            DCopy dc;
            dcopy_load<NT>(pd.du64, pd.outD, sBlk, kDChunks, stp, wave, lane, dc);
            dcopy_store(dc, lane);
        }
    }
}

// One member tile (item) of one problem; sTile, sBlk, sTerm, sW and sU are the
// workgroup's LDS tables and staging buffers.
template <int NP, bool WD>
__device__ __forceinline__ void class_bf16_item(const ProblemDescB &pd, int item, int32_t *sTile, int32_t *sBlk,
                                                int32_t *sTerm, u16x8 *sW, floatx4 *sU) {
    const int groups = pd.mtiles[4 * item + 2];
    if (groups == 0) return;            // an empty slot of a dispatch table
    if (groups == 4) class_bf16_tile<NP, 4, WD>(pd, item, sTile, sBlk, sTerm, sW, sU);
    else if (groups == 2) class_bf16_tile<NP, 2, WD>(pd, item, sTile, sBlk, sTerm, sW, sU);
    else class_bf16_tile<NP, 1, WD>(pd, item, sTile, sBlk, sTerm, sW, sU);
}

template <int NP, bool WD>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_class_bf16(ProblemDescB pd) {
    __shared__ int32_t sTile[64 * kTileStride];
    __shared__ int32_t sBlk[128];                    // stored block per member row; D-hat source block
    __shared__ int32_t sTerm[2 * kMaxClassTerms];     // unique-block pairs of the class
    __shared__ u16x8 sW[4 * NP * 64 * 4];            // staged W, four buffers
    __shared__ floatx4 sU[4 * 512];                  // staged B_IK values, four buffers
    class_bf16_item<NP, WD>(pd, blockIdx.x, sTile, sBlk, sTerm, sW, sU);
}

// Many problems in one persistent launch, split BF16 (the queues and their
// draining as in k_batch_f32; one 8-wave workgroup per CU).
template <int NP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_batch_bf16(const ProblemDescB *__restrict__ probs, const int32_t *__restrict__ items,
                  const int32_t *__restrict__ qb, int32_t nq, int32_t *__restrict__ counters) {
    __shared__ int32_t sTile[64 * kTileStride];
    __shared__ int32_t sBlk[128];
    __shared__ int32_t sTerm[2 * kMaxClassTerms];
    __shared__ u16x8 sW[4 * NP * 64 * 4];
    __shared__ floatx4 sU[4 * 512];
    __shared__ int32_t sItem;
    const int home = blockIdx.x % nq;
    int tried = 0;                       // queues found empty (thread 0)
    for (;;) {
        if (threadIdx.x == 0) sItem = batch_next_item(qb, nq, counters, home, tried);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(sItem);   // uniform: descriptors in scalar registers
        __syncthreads();                 // every thread has read sItem before it changes
        if (it < 0) break;
        const ProblemDescB pd = probs[items[2 * it]];
        class_bf16_item<NP, false>(pd, items[2 * it + 1], sTile, sBlk, sTerm, sW, sU);
    }
}

// Scratch of the allocation-free entry point: N^-1 in the MFMA operand format
// (three BF16 parts or FP32) for up to kNoAllocMaxPix pixels.  Each device
// that loads this code object holds one copy until the process ends.
static __device__ __align__(256) uint16_t scratch[3 * kNoAllocMaxPix];

}  // namespace

hipError_t noalloc_scratch(int device, void **ptr) {
    // the array's name is a host-side stand-in: its device address comes from
    // the runtime, once per device, with that device current
    static std::mutex mu;
    static void *addr[kNoAllocMaxDevices] = {};
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_tabulate(const double *coef, int32_t lmax, double h, double *table,
                           int32_t n_nodes, hipStream_t st) {
    const int threads = 256;
    const int blocks = (n_nodes + threads - 1) / threads;
    hipLaunchKernelGGL(k_tabulate, dim3(blocks), dim3(threads), 0, st, coef, lmax, h, table, n_nodes);
    return hipGetLastError();
}

hipError_t launch_eval(KTable kt, const double *y, double *out, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_eval, dim3((unsigned)blocks), dim3(256), 0, st, kt, y, out, n);
    return hipGetLastError();
}

hipError_t launch_unique_eval(KTable kt, const UInfo *uinfo, int64_t nunique, const double *ring_theta,
                              const double *ring_sin, double *u64, double *u64t, float *ut32, hipStream_t st) {
    if (nunique == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unique_eval, dim3((unsigned)nunique), dim3(256), 0, st, kt, uinfo, ring_theta,
                       ring_sin, u64, u64t, ut32);
    return hipGetLastError();
}

hipError_t launch_expand(const double *u64, const int32_t *items, int64_t nitems, const int32_t *exp_blk,
                         double *out, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3((unsigned)nitems), dim3(256), 0, st, u64, items, exp_blk, out);
    return hipGetLastError();
}

hipError_t launch_btnb(int prec, const BtnbArgs &a, hipStream_t st) {
    if (a.nblocks == 0) return hipSuccess;
    if (prec == 0) {
        ProblemDesc64 pd{a.mtiles, a.classes, a.class_terms, a.class_blk, a.class_itab, a.u64t, a.ninv, a.out,
                         a.du64, a.blk_uid, a.outD};
        if (a.outD) hipLaunchKernelGGL(k_class_f64<true>, dim3((unsigned)a.nmtiles), dim3(256), 0, st, pd);
        else hipLaunchKernelGGL(k_class_f64<false>, dim3((unsigned)a.nmtiles), dim3(256), 0, st, pd);
        return hipGetLastError();
    }
    if (prec == 1) {
        hipLaunchKernelGGL(k_ninv_f32, dim3((unsigned)((a.npix + 255) / 256)), dim3(256), 0, st, a.ninv,
                           a.npix, a.wf32);
        ProblemDesc pd{a.mtiles, a.classes, a.class_terms, a.class_blk, a.class_itab, a.ut32, a.wf32, a.out,
                       a.du64, a.blk_uid, a.outD};
        if (a.outD) hipLaunchKernelGGL(k_class_f32<true>, dim3((unsigned)a.nmtiles), dim3(512), 0, st, pd);
        else hipLaunchKernelGGL(k_class_f32<false>, dim3((unsigned)a.nmtiles), dim3(512), 0, st, pd);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_split_ninv, dim3((unsigned)((a.npix + 255) / 256)), dim3(256), 0, st, a.ninv,
                       a.npix, a.wsplit[0], a.wsplit[1], a.wsplit[2]);
    const dim3 grid((unsigned)a.nmtiles);
    ProblemDescB pd{a.mtiles, a.classes, a.class_terms, a.class_blk, a.class_itab, a.ut32,
                    {a.wsplit[0], a.wsplit[1], a.wsplit[2]}, a.out, a.du64, a.blk_uid, a.outD};
    if (a.outD) {
        if (prec == 2) hipLaunchKernelGGL((k_class_bf16<2, true>), grid, dim3(512), 0, st, pd);
        else hipLaunchKernelGGL((k_class_bf16<3, true>), grid, dim3(512), 0, st, pd);
    } else {
        if (prec == 2) hipLaunchKernelGGL((k_class_bf16<2, false>), grid, dim3(512), 0, st, pd);
        else hipLaunchKernelGGL((k_class_bf16<3, false>), grid, dim3(512), 0, st, pd);
    }
    return hipGetLastError();
}

hipError_t launch_batch(const BatchLaunch &b, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, b.counters, b.nq, 0);
    if (b.prec == 0) {                   // FP64: N^-1 is read as given
        if (b.persistent) {
            if (b.nitems > 0)
                hipLaunchKernelGGL(k_batch_f64, dim3((unsigned)b.nworkgroups), dim3(256), 0, st, b.desc64, b.items,
                                   b.qb, b.nq, b.counters);
        } else {
            for (int p = 0; p < b.nprob; ++p) {
                if (b.ngtiles[p] == 0) continue;
                ProblemDesc64 d = b.host_desc64[p];
                d.mtiles = b.gtiles[p];
                hipLaunchKernelGGL(k_class_f64<false>, dim3((unsigned)b.ngtiles[p]), dim3(256), 0, st, d);
            }
        }
        return hipGetLastError();
    }
    const bool bf16 = b.prec != 1;
    for (int p = 0; p < b.nprob; ++p) {
        if (b.npix[p] == 0) continue;
        const dim3 g((unsigned)((b.npix[p] + 255) / 256));
        if (!bf16) {
            hipLaunchKernelGGL(k_ninv_f32, g, dim3(256), 0, st, b.ninv[p], b.npix[p], b.host_desc[p].wf);
        } else {
            uint16_t *const *w = b.wsplit + 3 * p;
            hipLaunchKernelGGL(k_split_ninv, g, dim3(256), 0, st, b.ninv[p], b.npix[p], w[0], w[1], w[2]);
        }
    }
    if (b.persistent) {
        if (b.nitems > 0) {
            const dim3 g((unsigned)b.nworkgroups);
            if (!bf16)
                hipLaunchKernelGGL(k_batch_f32, g, dim3(512), 0, st, b.desc, b.items, b.qb, b.nq, b.counters);
            else if (b.prec == 2)
                hipLaunchKernelGGL(k_batch_bf16<2>, g, dim3(512), 0, st, b.descb, b.items, b.qb, b.nq, b.counters);
            else
                hipLaunchKernelGGL(k_batch_bf16<3>, g, dim3(512), 0, st, b.descb, b.items, b.qb, b.nq, b.counters);
        }
    } else {
        for (int p = 0; p < b.nprob; ++p) {
            if (b.ngtiles[p] == 0) continue;
            const dim3 g((unsigned)b.ngtiles[p]);
            if (!bf16) {
                ProblemDesc d = b.host_desc[p];
                d.mtiles = b.gtiles[p];
                hipLaunchKernelGGL(k_class_f32<false>, g, dim3(512), 0, st, d);
            } else {
                ProblemDescB d = b.host_descb[p];
                d.mtiles = b.gtiles[p];
                if (b.prec == 2) hipLaunchKernelGGL((k_class_bf16<2, false>), g, dim3(512), 0, st, d);
                else hipLaunchKernelGGL((k_class_bf16<3, false>), g, dim3(512), 0, st, d);
            }
        }
    }
    return hipGetLastError();
}

hipError_t batch_occupancy(int prec, int *workgroups_per_cu) {
    if (prec == 0) return hipOccupancyMaxActiveBlocksPerMultiprocessor(workgroups_per_cu, k_batch_f64, 256, 0);
    if (prec == 1) return hipOccupancyMaxActiveBlocksPerMultiprocessor(workgroups_per_cu, k_batch_f32, 512, 0);
    if (prec == 2) return hipOccupancyMaxActiveBlocksPerMultiprocessor(workgroups_per_cu, k_batch_bf16<2>, 512, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(workgroups_per_cu, k_batch_bf16<3>, 512, 0);
}

hipError_t launch_convolve(const double *u64, const int32_t *chunks, int64_t nchunks, const int32_t *slots,
                           const double *f, double *g, hipStream_t st) {
    if (nchunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_convolve, dim3((unsigned)nchunks), dim3(256), 0, st, u64, chunks, slots, f, g);
    return hipGetLastError();
}

}  // namespace sympix
