// Block-Jacobi preconditioner of the system matrix D-hat + B-hat^T N^-1 B-hat
// (gfx950): for every tile J, the Cholesky factor of its diagonal block
// A_J = D_JJ + C_JJ, and the application x_J = A_J^-1 r_J.
//
//   k_factor_diag  one wave per tile.  Lane l holds column l of A_J's upper
//                  triangle (64 doubles in registers, read row by row with
//                  coalesced 512-byte loads), i.e. row l of the lower factor
//                  being built.  Step j takes the pivot from lane j, scales
//                  column j (a multiply by the pivot's reciprocal, as
//                  LAPACK's unblocked factorisation does), passes it through
//                  LDS and updates the trailing rows: 64 sequential steps,
//                  about 2,000 FMAs per lane, no workgroup barrier.
//   k_solve_diag   one wave per tile, column l of U in lane l's registers:
//                  U^T y = r as a column sweep (lane l accumulates row l),
//                  then U x = y as a column sweep from the last row, whose
//                  columns reach the other lanes through LDS eight at a time.
//                  Both multiply by the reciprocals of U's diagonal.
//
// Both are bound by HBM: the factor reads two 32 KiB blocks and writes one
// per tile, the solve reads one and 1 KiB of vectors.
#include <hip/hip_runtime.h>

#include "precond.hpp"

namespace sympix {
namespace {

constexpr int kN = 64;       // pixels per tile (k = 8)
constexpr int kWaves = 4;    // tiles per workgroup, one wave each

// v as held by lane `src` (a constant of the unrolled loops), in every lane.
__device__ __forceinline__ double from_lane(double v, int src) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <bool WITH_C>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(3))) void k_factor_diag(const double *__restrict__ D,
                                                             const double *__restrict__ C,
                                                             const int32_t *__restrict__ dblk, int64_t ntiles,
                                                             double *__restrict__ U, int32_t *__restrict__ info) {
    __shared__ double sCol[kWaves][2][kN];   // the scaled column of a step, two buffers per wave
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t J = (int64_t)blockIdx.x * kWaves + wave;
    if (J >= ntiles) return;                 // the whole wave
    const int64_t base = (int64_t)dblk[J] * (kN * kN);
    double u[kN];                            // u[c] = A[c][lane]: upper triangle for c <= lane
#pragma unroll
    for (int c0 = 0; c0 < kN; c0 += 8) {    // eight rows at a time: D and C rows in flight together
        double t[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            u[c0 + c] = D[base + (c0 + c) * kN + lane];
            if constexpr (WITH_C) t[c] = C[base + (c0 + c) * kN + lane];
        }
        if constexpr (WITH_C) {
#pragma unroll
            for (int c = 0; c < 8; ++c) u[c0 + c] += t[c];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    int bad = 0;
#pragma clang loop unroll(full)
    for (int j = 0; j < kN; ++j) {
        const double pivot = from_lane(u[j], j);   // A_jj less the earlier steps' updates
        if (bad == 0 && !(pivot > 0.0)) bad = j + 1;
        const double s = sqrt(pivot);
        const double inv = 1.0 / s;
        const double lj = lane == j ? s : (lane > j ? u[j] * inv : u[j]);   // L[lane][j]
        u[j] = lj;
        double *col = sCol[wave][j & 1];
        col[lane] = lj;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // A[lane][c] -= L[lane][j] L[c][j] for the rows below j, eight columns at a time; the
        // rows above take a zero multiplier instead of a branch, which would make the
        // register allocator keep copies of u
        const double m = lane > j ? -lj : 0.0;
#pragma unroll
        for (int c0 = j + 1; c0 < kN; c0 += 8) {
            double v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (c0 + t < kN) v[t] = col[c0 + t];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (c0 + t < kN) u[c0 + t] = fma(m, v[t], u[c0 + t]);
            __builtin_amdgcn_sched_barrier(0);   // keeps the LDS reads of later chunks from piling up
        }
    }
    double *out = U + J * (kN * kN);
#pragma unroll
    for (int c0 = 0; c0 < kN; c0 += 16) {   // U[c][lane] = L[lane][c], zero below the diagonal
#pragma unroll
        for (int c = c0; c < c0 + 16; ++c) out[c * kN + lane] = c <= lane ? u[c] : 0.0;
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lane == 0) info[J] = bad;
}

// r and x may be the same array: a wave reads its tile of r before it writes
// that tile of x.
__global__ __launch_bounds__(64 * kWaves) void k_solve_diag(const double *__restrict__ U, const double *r,
                                                            double *x, int64_t ntiles) {
    __shared__ double sT[kWaves][8][kN];     // eight columns of U: one block of back-substitution steps
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t J = (int64_t)blockIdx.x * kWaves + wave;
    if (J >= ntiles) return;
    const double *ut = U + J * (kN * kN);
    double u[kN];                            // u[c] = U[c][lane]
#pragma unroll
    for (int c = 0; c < kN; ++c) u[c] = ut[c * kN + lane];
    const double rinv = 1.0 / ut[lane * kN + lane];   // 1 / U[lane][lane]
    double z = r[J * kN + lane];
    // U^T y = r, a column sweep: row l of U^T is column l of U, held by lane l
#pragma unroll
    for (int c = 0; c < kN; ++c) {
        const double yc = from_lane(z, c) * from_lane(rinv, c);
        const double m = lane > c ? yc : 0.0;
        z = lane == c ? yc : fma(-u[c], m, z);
    }
    // U x = y, a column sweep from the last row: step i needs U[c][i] in lane c, i.e.
    // column i of U, held by lane i; eight steps at a time take their columns from LDS
    double xv = 0.0;
#pragma unroll
    for (int b = kN / 8 - 1; b >= 0; --b) {
        const int i0 = 8 * b;
        if (lane >= i0 && lane < i0 + 8) {   // rows c < i0 + 8 are the ones these steps update
            double *row = sT[wave][lane - i0];
#pragma unroll
            for (int c = 0; c < i0 + 8; c += 2) *reinterpret_cast<double2 *>(row + c) = make_double2(u[c], u[c + 1]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int i = i0 + 7; i >= i0; --i) {
            const double xi = from_lane(z, i) * from_lane(rinv, i);
            if (lane == i) xv = xi;
            const double m = lane < i ? xi : 0.0;
            z = fma(-sT[wave][i - i0][lane], m, z);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    x[J * kN + lane] = xv;
}

}  // namespace

hipError_t launch_factor_diag(const double *D, const double *C, const int32_t *dblk, int64_t ntiles, double *U,
                              int32_t *info, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    const int64_t blocks = (ntiles + kWaves - 1) / kWaves;
    if (C) hipLaunchKernelGGL(k_factor_diag<true>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, st, D, C, dblk, ntiles, U, info);
    else hipLaunchKernelGGL(k_factor_diag<false>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, st, D, C, dblk, ntiles, U, info);
    return hipGetLastError();
}

hipError_t launch_solve_diag(const double *U, const double *r, double *x, int64_t ntiles, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    const int64_t blocks = (ntiles + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(k_solve_diag, dim3((unsigned)blocks), dim3(64 * kWaves), 0, st, U, r, x, ntiles);
    return hipGetLastError();
}

}  // namespace sympix
