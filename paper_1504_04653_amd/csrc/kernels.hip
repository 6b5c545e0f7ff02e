// HIP kernels for SymPix local-operator sampling on gfx950 (CDNA4, wave64).
//
//   k_tabulate     kernel table of Eq. 10, FP64 Legendre recurrence in y
//   k_eval         table lookups at arbitrary y (interpolation tests)
//   k_unique_eval  one workgroup per unique block (Section 2.3 symmetry keys):
//                  pair geometry, table lookup, radial cut; writes FP64
//                  row-major and FP32 / BF16-split copies transposed via LDS
//   k_expand       D-hat: streams each stored block from its unique block
//   k_btnb_*       B-hat^T N^-1 B-hat (Eq. 15): one output block per wave (FP64)
//                  or per wave pair (FP32, split BF16), MFMA over the 64 pixels
//                  of each contraction tile, FP64 accumulation across tiles.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sympix {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)

// ---------------------------------------------------------------------------
// a6: kernel table.  Node i holds b at s = |i - 1| h, y = s^2 (node 0 mirrors
// node 2: the kernel is even in s).  Recurrence in y with D_l = P_l - P_{l-1}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tabulate(const double *__restrict__ coef, int lmax,
                                                  double h, double *__restrict__ table,
                                                  int n_nodes) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const double s = (double)(i > 0 ? i - 1 : 1) * h;
    const double y = s * s;
    double p = 1.0;
    double acc = coef[0] * kInv4Pi;
    double d = -y;
    for (int l = 0; l < lmax; ++l) {
        if (l > 0) d = ((double)l * d - (double)(2 * l + 1) * y * p) / (double)(l + 1);
        p = p + d;
        acc += (double)(2 * l + 3) * coef[l + 1] * kInv4Pi * p;
    }
    table[i] = acc;
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
                                                     float *__restrict__ ut32,
                                                     uint16_t *__restrict__ ubf_hi,
                                                     uint16_t *__restrict__ ubf_mid,
                                                     uint16_t *__restrict__ ubf_lo) {
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
        ut32[base + e] = (float)v;
        const uint16_t h = bf16_bits((float)v);
        const double r1 = v - (double)bf16_value(h);
        const uint16_t m = bf16_bits((float)r1);
        const double r2 = r1 - (double)bf16_value(m);
        ubf_hi[base + e] = h;
        ubf_mid[base + e] = m;
        ubf_lo[base + e] = bf16_bits((float)r2);
    }
}

// ---------------------------------------------------------------------------
// a8: D-hat expansion.  Each stored block is a 32 KiB copy of its unique block,
// streamed with 16-byte non-temporal stores.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_expand(const double *__restrict__ u64,
                                                const int32_t *__restrict__ blk_uid,
                                                int64_t nblocks, double *__restrict__ out) {
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const doublex2 *src = (const doublex2 *)(u64 + (int64_t)blk_uid[b] * kBlockElems);
        doublex2 *dst = (doublex2 *)(out + b * kBlockElems);
        doublex2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = src[threadIdx.x + 256 * j];
#pragma unroll
        for (int j = 0; j < 8; ++j) __builtin_nontemporal_store(v[j], &dst[threadIdx.x + 256 * j]);
    }
}

// ---------------------------------------------------------------------------
// a9, FP64: one wave per output block C_JK (64 x 64), 16 MFMA 16x16x4 tiles
// per wave.  For a term I: A = B_IJ (rows p in I, cols a in J), B = B_IK, and
// C[a][b] += sum_p A[p][a] w_p B[p][b].  MFMA operand lanes: A fragment holds
// (row a = 16 i + lane%16, k = p), B fragment (k = p, col b = 16 j + lane%16),
// with p = 4 ks + lane/16.  The FP64 result interleaves rows: lane holds rows
// lane/16 + 4 v of column lane%16 (the FP32/BF16 16x16 forms hold 4 (lane/16) + v).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_btnb_f64(const double *__restrict__ u64,
                                                  const int64_t *__restrict__ term_ptr,
                                                  const DevTerm *__restrict__ terms,
                                                  const double *__restrict__ ninv,
                                                  int64_t nblocks, double *__restrict__ out) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 4 + wave;
    if (blk >= nblocks) return;
    const int lr = lane & 15, lk = lane >> 4;
    doublex4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    const int64_t t0 = term_ptr[blk], t1 = term_ptr[blk + 1];
    for (int64_t t = t0; t < t1; ++t) {
        const DevTerm tm = terms[t];
        const double *A = u64 + (int64_t)tm.uid_a * kBlockElems + lr;
        const double *B = u64 + (int64_t)tm.uid_b * kBlockElems + lr;
        const double *w = ninv + (int64_t)tm.tile * 64;
#pragma unroll 2
        for (int ks = 0; ks < 16; ++ks) {
            const int p = ks * 4 + lk;
            const double wp = w[p];
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = A[p * 64 + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = B[p * 64 + 16 * j] * wp;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    double *o = out + blk * kBlockElems + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                __builtin_nontemporal_store(acc[i][j][v], &o[(16 * i + lk + 4 * v) * 64 + 16 * j]);
}

// ---------------------------------------------------------------------------
// a9, FP32 MFMA: two waves per output block (columns 0-31 / 32-63).  Operands
// are rounded to FP32 after folding w_p into B in FP64; each term's 64-pixel
// sum runs in the FP32 MFMA accumulator and is added to FP64 accumulators.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_btnb_f32(const double *__restrict__ u64,
                                                  const int64_t *__restrict__ term_ptr,
                                                  const DevTerm *__restrict__ terms,
                                                  const double *__restrict__ ninv,
                                                  int64_t nblocks, double *__restrict__ out) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 2 + (wave >> 1);
    const int half = wave & 1;
    if (blk >= nblocks) return;
    const int lr = lane & 15, lk = lane >> 4;
    doublex4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    const int64_t t0 = term_ptr[blk], t1 = term_ptr[blk + 1];
    for (int64_t t = t0; t < t1; ++t) {
        const DevTerm tm = terms[t];
        const double *A = u64 + (int64_t)tm.uid_a * kBlockElems + lr;
        const double *B = u64 + (int64_t)tm.uid_b * kBlockElems + 32 * half + lr;
        const double *w = ninv + (int64_t)tm.tile * 64;
        floatx4 part[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) part[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
            const int p = ks * 4 + lk;
            const double wp = w[p];
            float a[4], b[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = (float)A[p * 64 + 16 * i];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = (float)(B[p * 64 + 16 * j] * wp);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], part[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)part[i][j][v];
    }
    double *o = out + blk * kBlockElems + 32 * half + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                __builtin_nontemporal_store(acc[i][j][v], &o[(16 * i + 4 * lk + v) * 64 + 16 * j]);
}

// ---------------------------------------------------------------------------
// a9, split BF16: two waves per output block.  A = B_IJ comes pre-split (FP64
// value into 3 BF16 parts, transposed so a lane's 8 consecutive p are one
// 16-byte load); B = w_p B_IK is formed in FP32 from the FP32 copy and split
// on the fly (three BF16 parts of an FP32 value are exact).  MFMA 16x16x32
// BF16 with FP32 accumulation per term, FP64 across terms.  NPARTS = 2 uses
// hi*hi + hi*mid + mid*hi; NPARTS = 3 adds hi*lo + lo*hi + mid*mid.
// ---------------------------------------------------------------------------
template <int NPARTS>
__global__ __launch_bounds__(256) void k_btnb_bf16(const uint16_t *__restrict__ ubf_hi,
                                                   const uint16_t *__restrict__ ubf_mid,
                                                   const uint16_t *__restrict__ ubf_lo,
                                                   const float *__restrict__ ut32,
                                                   const int64_t *__restrict__ term_ptr,
                                                   const DevTerm *__restrict__ terms,
                                                   const double *__restrict__ ninv,
                                                   int64_t nblocks, double *__restrict__ out) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 2 + (wave >> 1);
    const int half = wave & 1;
    if (blk >= nblocks) return;
    const int lr = lane & 15, lk = lane >> 4;
    doublex4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    const int64_t t0 = term_ptr[blk], t1 = term_ptr[blk + 1];
    for (int64_t t = t0; t < t1; ++t) {
        const DevTerm tm = terms[t];
        const int64_t abase = (int64_t)tm.uid_a * kBlockElems + lr * 64 + 8 * lk;
        const int64_t bbase = (int64_t)tm.uid_b * kBlockElems + (32 * half + lr) * 64 + 8 * lk;
        const double *w = ninv + (int64_t)tm.tile * 64 + 8 * lk;
        floatx4 part[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) part[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int p0 = 32 * ks;
            float wf[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) wf[e] = (float)w[p0 + e];
            bf16x8 bh[2], bm[2], bl[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const floatx4 *src = (const floatx4 *)(ut32 + bbase + 16 * j * 64 + p0);
                const floatx4 u0 = src[0], u1 = src[1];
                u16x8 h, m, l;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float x = wf[e] * (e < 4 ? u0[e] : u1[e - 4]);
                    const uint16_t hb = bf16_bits(x);
                    const float r1 = x - bf16_value(hb);
                    const uint16_t mb = bf16_bits(r1);
                    h[e] = hb;
                    m[e] = mb;
                    if (NPARTS == 3) l[e] = bf16_bits(r1 - bf16_value(mb));
                }
                bh[j] = __builtin_bit_cast(bf16x8, h);
                bm[j] = __builtin_bit_cast(bf16x8, m);
                if (NPARTS == 3) bl[j] = __builtin_bit_cast(bf16x8, l);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t off = abase + 16 * i * 64 + p0;
                const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const u16x8 *)(ubf_hi + off));
                const bf16x8 am = __builtin_bit_cast(bf16x8, *(const u16x8 *)(ubf_mid + off));
                bf16x8 al;
                if (NPARTS == 3) al = __builtin_bit_cast(bf16x8, *(const u16x8 *)(ubf_lo + off));
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    floatx4 c = part[i][j];
                    if (NPARTS == 3) {
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm[j], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], c, 0, 0, 0);
                    }
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[j], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[j], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], c, 0, 0, 0);
                    part[i][j] = c;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)part[i][j][v];
    }
    double *o = out + blk * kBlockElems + 32 * half + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                __builtin_nontemporal_store(acc[i][j][v], &o[(16 * i + 4 * lk + v) * 64 + 16 * j]);
}

}  // namespace

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

hipError_t launch_unique_eval(KTable kt, const UInfo *uinfo, int64_t nunique, int32_t k,
                              const double *ring_theta, const double *ring_sin, double *u64,
                              float *ut32, uint16_t *ubf_hi, uint16_t *ubf_mid, uint16_t *ubf_lo,
                              hipStream_t st) {
    (void)k;
    if (nunique == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unique_eval, dim3((unsigned)nunique), dim3(256), 0, st, kt, uinfo,
                       ring_theta, ring_sin, u64, ut32, ubf_hi, ubf_mid, ubf_lo);
    return hipGetLastError();
}

hipError_t launch_expand(const double *u64, const int32_t *blk_uid, int64_t nblocks, double *out,
                         hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const int64_t grid = nblocks < 4096 ? nblocks : 4096;
    hipLaunchKernelGGL(k_expand, dim3((unsigned)grid), dim3(256), 0, st, u64, blk_uid, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_btnb(int prec, const double *u64, const float *ut32, const uint16_t *ubf_hi,
                       const uint16_t *ubf_mid, const uint16_t *ubf_lo, const int64_t *term_ptr,
                       const DevTerm *terms, const double *ninv, int64_t nblocks, double *out,
                       hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (prec == 0) {
        const int64_t grid = (nblocks + 3) / 4;
        hipLaunchKernelGGL(k_btnb_f64, dim3((unsigned)grid), dim3(256), 0, st, u64, term_ptr,
                           terms, ninv, nblocks, out);
    } else {
        const int64_t grid = (nblocks + 1) / 2;
        if (prec == 1)
            hipLaunchKernelGGL(k_btnb_f32, dim3((unsigned)grid), dim3(256), 0, st, u64, term_ptr,
                               terms, ninv, nblocks, out);
        else if (prec == 2)
            hipLaunchKernelGGL(k_btnb_bf16<2>, dim3((unsigned)grid), dim3(256), 0, st, ubf_hi,
                               ubf_mid, ubf_lo, ut32, term_ptr, terms, ninv, nblocks, out);
        else
            hipLaunchKernelGGL(k_btnb_bf16<3>, dim3((unsigned)grid), dim3(256), 0, st, ubf_hi,
                               ubf_mid, ubf_lo, ut32, term_ptr, terms, ninv, nblocks, out);
    }
    return hipGetLastError();
}

}  // namespace sympix
