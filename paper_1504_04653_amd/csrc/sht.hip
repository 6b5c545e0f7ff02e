// Spherical harmonic transforms on the SymPix geometry (gfx950): synthesis
// f = Y a, its transpose Y^T f, the quadrature analysis Y^T W f of Eq. 1 and,
// built from them, the degrade theta_2 = W_2 Y_2 Y_obs^T theta of Eq. 14.
//
// Real orthonormal harmonics without the Condon-Shortley phase: Y_{l,0} =
// lambda_l0, Y_{l,+-m} = sqrt(2) lambda_lm cos / sin(m phi).  A transform
// splits into a Legendre part per m (over all rings, O(L^2 N_ring)) and a
// Fourier part per ring (O(n log n)):
//
//   k_alm_mm   the coefficient vector to m-major rows (and back)
//   k_leg_syn  one workgroup per m: F_m(ring) = sum_l a_lm lambda_lm(theta),
//              north and south rings of a pair together (lambda_lm(pi - t) =
//              (-1)^(l-m) lambda_lm(t): even and odd l - m summed apart)
//   k_ring_syn one workgroup per ring: the modes folded onto the ring's n
//              frequencies, an FFT in LDS (of length n / 2 for even n: the
//              ring's real values in pairs), the ring scattered to SymPix order
//   k_ring_adj the transpose: gather, FFT, unfold to the modes m <= L
//   k_leg_adj  one workgroup per m: a_lm = sum_rings lambda_lm G_m(ring),
//              reduced across the workgroup eight degrees at a time
//
// lambda_lm is carried from lambda_mm (tabulated on the host) by the monic
// form of its three-term recurrence in l, with a per-ring power-of-two scale
// (the recurrence section below).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sht.hpp"

namespace sympix {
namespace {

constexpr int kRingThreads = 1024;   // ring kernels: one workgroup of 16 waves per ring
constexpr int kLegThreads = 256;     // Legendre kernels
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kBig = 0x1p300, kSmall = 0x1p-300;

// ---------------------------------------------------------------------------
// Coefficient layout: (L+1)^2 entries at l^2 + l + m  <->  m-major rows (row
// m from row_off[m], entry i = l - m, zero padding after entry L - m) of cos
// (m >= 0) and sin (m >= 1; the m = 0 row is zero) coefficients, each held
// times K_lm, the scale of the monic recurrence below.
// ---------------------------------------------------------------------------
// Layout changes between the two orders, tiled (32 orders x 32 degrees per
// workgroup of 256 threads) and transposed through LDS, so that the vector
// (consecutive m at one l) and the rows (consecutive l at one m) are both read
// and written in runs.  Tiles holding no l >= m exit at once.
constexpr int kMmTile = 32;

template <bool TO_MM>
__global__ __launch_bounds__(256) void k_alm_mm(const double *__restrict__ src, int L,
                                                const int64_t *__restrict__ row_off,
                                                const double *__restrict__ rk, double *__restrict__ ac,
                                                double *__restrict__ as, double *__restrict__ dst) {
    __shared__ double tc[kMmTile][kMmTile + 1], ts[kMmTile][kMmTile + 1];   // [m - m0][l - l0]
    const int m0 = blockIdx.y * kMmTile, l0 = blockIdx.x * kMmTile;
    if (l0 + kMmTile - 1 < m0) return;
    const int fast = threadIdx.x & 31, slow = threadIdx.x >> 5;
    if constexpr (TO_MM) {
        for (int q = slow; q < kMmTile; q += 8) {        // one degree per pass, consecutive m
            const int l = l0 + q, m = m0 + fast;
            if (l <= L && m <= l) {
                const int64_t c = (int64_t)l * l + l;
                tc[fast][q] = src[c + m];
                ts[fast][q] = m == 0 ? 0.0 : src[c - m];
            }
        }
        __syncthreads();
        for (int q = slow; q < kMmTile; q += 8) {        // one order per pass, consecutive l, times K
            const int m = m0 + q, l = l0 + fast;
            if (l <= L && m <= l) {
                const int64_t o = row_off[m] + l - m;
                const double k = rk[o];
                ac[o] = tc[q][fast] * k;
                as[o] = ts[q][fast] * k;
            }
        }
    } else {
        for (int q = slow; q < kMmTile; q += 8) {        // one order per pass, consecutive l, over K
            const int m = m0 + q, l = l0 + fast;
            if (l <= L && m <= l) {
                const int64_t o = row_off[m] + l - m;
                const double k = rk[o];
                tc[q][fast] = ac[o] / k;
                ts[q][fast] = as[o] / k;
            }
        }
        __syncthreads();
        for (int q = slow; q < kMmTile; q += 8) {        // one degree per pass, consecutive m
            const int l = l0 + q, m = m0 + fast;
            if (l <= L && m <= l) {
                const int64_t c = (int64_t)l * l + l;
                dst[c + m] = tc[fast][q];
                if (m > 0) dst[c - m] = ts[fast][q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The recurrence.  lambda_lm = 2^e K_i mu_i (i = l - m), where mu follows the
// monic recurrence mu_i = cos(theta) mu_{i-1} - b_i mu_{i-2} with b_i =
// ((l-1)^2 - m^2) / (4 (l-1)^2 - 1); b_0 = -1 starts it from (mu_{-1},
// mu_{-2}) = (0, lambda_mm 2^-e).  K_i is the product of the factors alpha_j
// = sqrt((4 l_j^2 - 1) / (l_j^2 - m^2)) of the normalised recurrence over j in
// [64 c, i], the 64-degree chunk c of i (j >= 1), so that K stays within the
// double range; at a chunk start mu_{i-1} and mu_{i-2} are multiplied by K of
// the chunk before's last degree.  A step is then one multiply and one fused
// multiply-add, and the per-degree values (b_i, the coefficients times K) are
// the same for every ring: the kernels read them with uniform loads, which go
// through the scalar cache into scalar registers.
//
// When |mu| has grown past 2^300 at a test (one per four or eight degrees),
// mu is scaled by 2^-300 and e raised by 300, so that the values far below the
// double range near the poles at high m still reach the degrees where they
// matter.  Between tests |mu| grows by less than 1.25 per degree (|cos| <= 1,
// 0 <= b_i < 1/4), and by at most 2^270 at a chunk start, so that it stays
// below 2^600.
// ---------------------------------------------------------------------------
// Workgroups go to the 8 XCDs in turn (workgroup w on XCD w mod 8).  The
// Legendre kernels' ring buffer holds, per ring, the orders m in 16-byte
// entries, so one 128-byte line holds 8 consecutive orders; the workgroups of
// those orders are put on one XCD, whose L2 then merges their entries:
// w = 8 (8 (g / 8) + m mod 8) + g mod 8 for m = 8 g + (m mod 8), the orders in
// increasing m (largest rows first) on every XCD; -1 past L.
constexpr int kXcds = 8;

__device__ __forceinline__ int order_of_workgroup(int L) {
    const int w = blockIdx.x, x = w % kXcds, s = w / kXcds;
    const int m = kXcds * (x + kXcds * (s / kXcds)) + s % kXcds;
    return m <= L ? m : -1;
}

__host__ __forceinline__ int order_workgroups(int L) {
    const int g = kXcds * kXcds;
    return (L + 1 + g - 1) / g * g;
}

struct Deg4 { double v[4]; };   // four consecutive degrees of a row (32-byte aligned)

__device__ __forceinline__ Deg4 deg4(const double *p) { return *(const Deg4 *)p; }

// ---------------------------------------------------------------------------
// Legendre synthesis.  Workgroup m; thread t takes the ring pairs t + 256 q
// (R of them at a time, interleaved for latency).  Degrees go four at a time
// (even, odd, even, odd i), the next four read ahead; the rescale test is made
// once per four degrees (four steps grow |mu| by less than 2.5).
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(kLegThreads) void k_leg_syn(ShtDesc d, const int64_t *__restrict__ row_off,
                                                         const double *__restrict__ rb,
                                                         const double *__restrict__ rk,
                                                         const double *__restrict__ ac,
                                                         const double *__restrict__ as,
                                                         double *__restrict__ fbuf) {
    const int m = order_of_workgroup(d.lmax);
    if (m < 0) return;
    const int L = d.lmax, nl = L - m + 1;
    const int64_t off = row_off[m];
    const double *b = rb + off, *kk = rk + off, *cc = ac + off, *cs = as + off;
    for (int rp0 = threadIdx.x; rp0 < d.nhalf; rp0 += kLegThreads * R) {
        double ct[R], mu[R], mup[R], ec[R], es[R], oc[R], os[R];
        int e[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int rp = min(rp0 + kLegThreads * q, d.nhalf - 1);
            ct[q] = d.ring_cos[rp];
            mu[q] = 0.0;
            mup[q] = d.lmm_mant[(int64_t)m * d.nhalf + rp];
            e[q] = d.lmm_exp[(int64_t)m * d.nhalf + rp];
            ec[q] = es[q] = oc[q] = os[q] = 0.0;
        }
        Deg4 gb = deg4(b), gc = deg4(cc), gs = deg4(cs);
        for (int i0 = 0; i0 < nl; i0 += 4) {
            const Deg4 nb = deg4(b + i0 + 4), nc = deg4(cc + i0 + 4), ns = deg4(cs + i0 + 4);
            if (i0 != 0 && (i0 & 63) == 0) {      // chunk start: carry K of the chunk before
                const double sk = kk[i0 - 1];
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    mu[q] *= sk;
                    mup[q] *= sk;
                }
            }
            // the test of all rings at once, one wave-uniform branch: short
            // per-ring branches would be executed under a mask every time
            bool grow = false;
#pragma unroll
            for (int q = 0; q < R; ++q) grow |= fabs(mu[q]) > kBig;
            if (__builtin_expect(__any(grow), 0)) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    if (fabs(mu[q]) > kBig) {
                        mu[q] *= kSmall;
                        mup[q] *= kSmall;
                        ec[q] *= kSmall;
                        es[q] *= kSmall;
                        oc[q] *= kSmall;
                        os[q] *= kSmall;
                        e[q] += 300;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double x0 = fma(ct[q], mu[q], -gb.v[0] * mup[q]);   // even i
                ec[q] = fma(gc.v[0], x0, ec[q]);
                es[q] = fma(gs.v[0], x0, es[q]);
                const double x1 = fma(ct[q], x0, -gb.v[1] * mu[q]);      // odd
                oc[q] = fma(gc.v[1], x1, oc[q]);
                os[q] = fma(gs.v[1], x1, os[q]);
                const double x2 = fma(ct[q], x1, -gb.v[2] * x0);         // even
                ec[q] = fma(gc.v[2], x2, ec[q]);
                es[q] = fma(gs.v[2], x2, es[q]);
                const double x3 = fma(ct[q], x2, -gb.v[3] * x1);         // odd
                oc[q] = fma(gc.v[3], x3, oc[q]);
                os[q] = fma(gs.v[3], x3, os[q]);
                mup[q] = x2;
                mu[q] = x3;
            }
            gb = nb;
            gc = nc;
            gs = ns;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int rp = rp0 + kLegThreads * q;
            if (rp >= d.nhalf) continue;
            const int rs = d.nrings - 1 - rp;
            double *fn = fbuf + ((int64_t)rp * (L + 1) + m) * 2;
            double *fs = fbuf + ((int64_t)rs * (L + 1) + m) * 2;
            fn[0] = ldexp(ec[q] + oc[q], e[q]);
            fn[1] = ldexp(es[q] + os[q], e[q]);
            fs[0] = ldexp(ec[q] - oc[q], e[q]);
            fs[1] = ldexp(es[q] - os[q], e[q]);
        }
    }
}

// ---------------------------------------------------------------------------
// Legendre transpose.  Workgroup m; thread t carries the ring pairs t + 256 q
// (q < R, R 256 >= nhalf), with G(north) +- G(south) scaled by 2^e, and adds
// mu_i times them over its rings, eight degrees at a time; the workgroup then
// sums the 256 partials of each of the 16 values (cos, sin x 8 degrees)
// through LDS and wave shuffles, and the result times K_i^2 (K_i for lambda,
// K_i for the stored scale) is written.  Degrees past L read b = 0 and are
// not written.
//
// While a ring's e is below kEMin its terms are left out: there |lambda| <
// 2^(e + 573) < 2^-387 (|mu| < 2^303 after a test, K < 2^270), far below the
// rounding of any sum.  2^e G would underflow there; when a rescale lifts e to
// kEMin or above, the ring's G is read again and scaled by the new 2^e.
// ---------------------------------------------------------------------------
constexpr int kEMin = -960;

struct RingG { double pc, mc, ps, ms; };

// G(north) +- G(south) of mode m on ring pair r, scaled by 2^e (zero below kEMin)
__device__ __forceinline__ RingG ring_g(const ShtDesc &d, const double *gbuf, int r, int m, int e) {
    const int L = d.lmax, rs = d.nrings - 1 - r;
    const double sc = e >= kEMin ? ldexp(1.0, e) : 0.0;
    const double *gn = gbuf + ((int64_t)r * (L + 1) + m) * 2;
    const double *gs = gbuf + ((int64_t)rs * (L + 1) + m) * 2;
    return RingG{(gn[0] + gs[0]) * sc, (gn[0] - gs[0]) * sc, (gn[1] + gs[1]) * sc, (gn[1] - gs[1]) * sc};
}

// up to six ring pairs per thread fit in 128 VGPRs (four waves per SIMD; the
// few values the compiler then keeps in scratch are read only on the rare
// reload path)
template <int T, int R>
__global__ __launch_bounds__(T, R <= 6 ? 4 : 1) void k_leg_adj(ShtDesc d, const int64_t *__restrict__ row_off,
                                                         const double *__restrict__ rb,
                                                         const double *__restrict__ rk,
                                                         const double *__restrict__ gbuf,
                                                         double *__restrict__ ac, double *__restrict__ as) {
    constexpr int CH = 8;
    constexpr int LPR = T / 16;          // lanes summing one of the 16 values
    __shared__ double sRed[2 * CH * T];
    const int m = order_of_workgroup(d.lmax);
    if (m < 0) return;
    const int L = d.lmax, nl = L - m + 1;
    const int64_t off = row_off[m];
    const double *b = rb + off, *kk = rk + off;
    double ct[R], mu[R], mup[R];
    RingG g[R];
    int e[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int rp = threadIdx.x + T * q;
        const bool ok = rp < d.nhalf;
        const int r = ok ? rp : 0;
        e[q] = d.lmm_exp[(int64_t)m * d.nhalf + r];
        ct[q] = d.ring_cos[r];
        mu[q] = 0.0;
        mup[q] = ok ? d.lmm_mant[(int64_t)m * d.nhalf + r] : 0.0;
        g[q] = ring_g(d, gbuf, r, m, e[q]);
    }
    Deg4 b0 = deg4(b), b1 = deg4(b + 4);
    for (int i0 = 0; i0 < nl; i0 += CH) {
        const Deg4 n0 = deg4(b + i0 + 8), n1 = deg4(b + i0 + 12);
        if (i0 != 0 && (i0 & 63) == 0) {
            const double sk = kk[i0 - 1];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                mu[q] *= sk;
                mup[q] *= sk;
            }
        }
        double vc[CH], vs[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) vc[j] = vs[j] = 0.0;
        bool grow = false;                 // as in the synthesis: one uniform branch
#pragma unroll
        for (int q = 0; q < R; ++q) grow |= fabs(mu[q]) > kBig;
        if (__builtin_expect(__any(grow), 0)) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (fabs(mu[q]) <= kBig) continue;
                mu[q] *= kSmall;
                mup[q] *= kSmall;
                e[q] += 300;
                if (e[q] - 300 >= kEMin) {
                    g[q].pc *= kBig;
                    g[q].mc *= kBig;
                    g[q].ps *= kBig;
                    g[q].ms *= kBig;
                } else if (e[q] >= kEMin) {       // the ring's terms start to count
                    // the ring index is made opaque, so that the compiler does not keep
                    // this rare reload's addresses live across the loop
                    int rr = min(threadIdx.x + T * q, d.nhalf - 1);
                    asm volatile("" : "+v"(rr));
                    g[q] = ring_g(d, gbuf, rr, m, e[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            double x = mu[q], xp = mup[q];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const double bj = j < 4 ? b0.v[j] : b1.v[j - 4];
                const double xn = fma(ct[q], x, -bj * xp);
                vc[j] = fma(xn, (j & 1) ? g[q].mc : g[q].pc, vc[j]);
                vs[j] = fma(xn, (j & 1) ? g[q].ms : g[q].ps, vs[j]);
                xp = x;
                x = xn;
            }
            mu[q] = x;
            mup[q] = xp;
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            sRed[j * T + threadIdx.x] = vc[j];
            sRed[(CH + j) * T + threadIdx.x] = vs[j];
        }
        __syncthreads();
        const int row = threadIdx.x / LPR, seg = threadIdx.x % LPR;
        double sum = 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) sum += sRed[row * T + t * LPR + seg];
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (seg == 0) {
            const int i = i0 + (row & (CH - 1));
            if (i < nl) {
                const double k2 = kk[i] * kk[i];
                if (row < CH) ac[off + i] = sum * k2;
                else as[off + i] = m == 0 ? 0.0 : sum * k2;
            }
        }
        __syncthreads();
        b0 = n0;
        b1 = n1;
    }
}

// ---------------------------------------------------------------------------
// FFT in LDS: forward DFT z_q <- sum_j z_j exp(-2 pi i j q / n) for n =
// 2^a 3^b 5^c <= kShtMaxRing, by self-sorting (Stockham) passes of radix 2,
// 3, 4 and 5.  Pass with radix R over sub-transforms of length Ns: butterfly
// j takes z[j + r n/R] (r < R), twiddles them by w^r, w = exp(-2 pi i (j mod
// Ns) / (Ns R)) (w from one sincospi, its powers by complex products: one or
// two roundings more), applies the R-point DFT and writes output r to (j / Ns) Ns R +
// (j mod Ns) + r Ns.  All reads of a pass precede all its writes (the
// workgroup holds the pass in registers between two barriers), so one buffer
// serves as input and output.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <int R>
__device__ __forceinline__ void dft_small(double2 *v) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = double2{a.x + b.x, a.y + b.y};
        v[1] = double2{a.x - b.x, a.y - b.y};
    } else if constexpr (R == 4) {
        const double2 s02 = double2{v[0].x + v[2].x, v[0].y + v[2].y};
        const double2 d02 = double2{v[0].x - v[2].x, v[0].y - v[2].y};
        const double2 s13 = double2{v[1].x + v[3].x, v[1].y + v[3].y};
        const double2 d13 = double2{v[1].x - v[3].x, v[1].y - v[3].y};
        v[0] = double2{s02.x + s13.x, s02.y + s13.y};
        v[2] = double2{s02.x - s13.x, s02.y - s13.y};
        v[1] = double2{d02.x + d13.y, d02.y - d13.x};    // d02 - i d13
        v[3] = double2{d02.x - d13.y, d02.y + d13.x};    // d02 + i d13
    } else if constexpr (R == 3) {
        constexpr double s3 = 0.86602540378443865;       // sqrt(3) / 2
        const double2 a = v[0], b = v[1], c = v[2];
        const double2 t = double2{b.x + c.x, b.y + c.y};
        const double2 u = double2{b.x - c.x, b.y - c.y};
        const double2 w = double2{a.x - 0.5 * t.x, a.y - 0.5 * t.y};
        v[0] = double2{a.x + t.x, a.y + t.y};
        v[1] = double2{w.x + s3 * u.y, w.y - s3 * u.x};  // w - i s3 u
        v[2] = double2{w.x - s3 * u.y, w.y + s3 * u.x};  // w + i s3 u
    } else {                                            // R == 5
        // cos and sin of 2 pi / 5 and 4 pi / 5
        constexpr double c1 = 0.30901699437494742, c2 = -0.80901699437494742;
        constexpr double s1 = 0.95105651629515357, s2 = 0.58778525229247313;
        const double2 a = v[0];
        const double2 t1 = double2{v[1].x + v[4].x, v[1].y + v[4].y};
        const double2 u1 = double2{v[1].x - v[4].x, v[1].y - v[4].y};
        const double2 t2 = double2{v[2].x + v[3].x, v[2].y + v[3].y};
        const double2 u2 = double2{v[2].x - v[3].x, v[2].y - v[3].y};
        const double2 w1 = double2{a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y};
        const double2 w2 = double2{a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y};
        const double2 q1 = double2{s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y};
        const double2 q2 = double2{s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y};
        v[0] = double2{a.x + t1.x + t2.x, a.y + t1.y + t2.y};
        v[1] = double2{w1.x + q1.y, w1.y - q1.x};        // w1 - i q1
        v[4] = double2{w1.x - q1.y, w1.y + q1.x};        // w1 + i q1
        v[2] = double2{w2.x + q2.y, w2.y - q2.x};        // w2 - i q2
        v[3] = double2{w2.x - q2.y, w2.y + q2.x};        // w2 + i q2
    }
}

template <int R, int MAXN>
__device__ __forceinline__ void fft_pass(double2 *z, int n, int Ns) {
    constexpr int MB = (MAXN / R + kRingThreads - 1) / kRingThreads;
    const int nb = n / R;
    double2 out[MB][R];
    int dst[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int j = threadIdx.x + kRingThreads * b;
        dst[b] = -1;
        if (j < nb) {
            const int k = j % Ns;
            double2 v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = z[j + r * nb];
            if (Ns > 1) {       // twiddles w^r, w = exp(-2 pi i k / (Ns R)): one sincos, then powers
                double sn, cs;
                sincospi(-2.0 * (double)k / (double)(Ns * R), &sn, &cs);
                const double2 w = double2{cs, sn};
                double2 wr = w;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    v[r] = cmul(v[r], wr);
                    if (r + 1 < R) wr = cmul(wr, w);
                }
            }
            dft_small<R>(v);
#pragma unroll
            for (int r = 0; r < R; ++r) out[b][r] = v[r];
            dst[b] = (j / Ns) * Ns * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MB; ++b)
        if (dst[b] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) z[dst[b] + r * Ns] = out[b][r];
        }
    __syncthreads();
}

template <int MAXN>
__device__ void fft_forward(double2 *z, int n, const int8_t *rad) {
    int Ns = 1;
    const int np = rad[0];
    for (int p = 1; p <= np; ++p) {
        const int R = rad[p];
        if (R == 4) fft_pass<4, MAXN>(z, n, Ns);
        else if (R == 2) fft_pass<2, MAXN>(z, n, Ns);
        else if (R == 3) fft_pass<3, MAXN>(z, n, Ns);
        else fft_pass<5, MAXN>(z, n, Ns);
        Ns *= R;
    }
}

// pixel of ring position j: tile j / k of the band, column j % k, this ring's
// row (folded into pix0)
__device__ __forceinline__ int64_t ring_pixel(const ShtDesc &d, int r, int j) {
    return d.ring_pix0[r] + (int64_t)(j / d.k) * d.k * d.k + (int64_t)(j % d.k) * d.k;
}

// Ring transforms.  A ring of even length n = 2N takes an FFT of length N
// (the ring's FFT length nf, whose radices the plan holds): its n real values
// pair up as N complex ones (x_2r + i x_2r+1), which halves the LDS and the
// butterflies.  A ring of odd length (odd tile sizes k) takes the FFT of
// length n.  MAXN bounds nf (the plan's longest), and sizes the registers one
// FFT pass holds.

// As for the orders above, and the k rings of a band interleave their pixels at a stride of k (one 128-byte line
// holds pixels of every ring of the band).  A band's rings are therefore given
// to workgroups on one XCD, w = 8 (k (band / 8) + row) + band mod 8, so that
// its L2 serves the shared lines; -1 past the last band.

__device__ __forceinline__ int ring_of_workgroup(const ShtDesc &d) {
    const int w = blockIdx.x, x = w % kXcds, s = w / kXcds;
    const int band = x + kXcds * (s / d.k), row = s % d.k;
    return band * d.k < d.nrings ? band * d.k + row : -1;
}

__host__ __forceinline__ int ring_workgroups(const ShtDesc &d) {
    const int nbands = d.nrings / d.k;
    return (nbands + kXcds - 1) / kXcds * kXcds * d.k;
}

// y_q = conj(sum_{m = q mod n, m <= L} H_m exp(i pi m / n)): the ring's modes
// H_0 = F_0, H_m = sqrt(2) (F_m^cos - i F_m^sin) folded onto frequency q with
// the half-pixel phase.  exp(i pi (q + j n) / n) = (-1)^j exp(i pi q / n), so
// the phase ph = exp(i pi q / n) is applied once, after the sum.
__device__ __forceinline__ double2 fold_mode(const double *F, int L, int n, int q, double2 ph) {
    double hr = 0.0, hi = 0.0, sg = 1.0;
    for (int m = q; m <= L; m += n) {
        const double hc = m == 0 ? F[0] : kSqrt2 * F[2 * m];
        const double hs = m == 0 ? 0.0 : -kSqrt2 * F[2 * m + 1];
        hr += sg * hc;
        hi += sg * hs;
        sg = -sg;
    }
    const double2 z = cmul(double2{hr, hi}, ph);
    return double2{z.x, -z.y};
}

// f_j = Re sum_m H_m exp(i m phi_j), phi_j = 2 pi (j + 1/2) / n, that is f =
// Re DFT_n(y).  Even n = 2N: with A_k = y_k + y_k+N and B_k = (y_k - y_k+N)
// w^k (w = exp(-2 pi i / n)), f_2r = Re DFT_N(A)_r and f_2r+1 = Re DFT_N(B)_r;
// taking the conjugate-even part of each, A'_k = (A_k + conj A_N-k) / 2 (and
// B'), makes both transforms real, so one FFT of C = A' + i B' gives f_2r +
// i f_2r+1.  A thread builds C_k and C_N-k together from y at k, k + N, N - k
// and n - k.  With wmul the ring is scaled by its pixel weight (W_2 of Eq. 14).
template <int MAXN>
__global__ __launch_bounds__(kRingThreads) void k_ring_syn(ShtDesc d, const double *__restrict__ fbuf,
                                                          double *__restrict__ map, int wmul) {
    extern __shared__ double2 z[];
    const int r = ring_of_workgroup(d);
    if (r < 0) return;
    const int L = d.lmax, n = d.ring_n[r];
    const double *F = fbuf + (int64_t)r * (L + 1) * 2;
    const double w = wmul ? d.ring_w[r] : 1.0;
    if (n & 1) {
        for (int k = threadIdx.x; k < n; k += kRingThreads) {
            double sn, cs;
            sincospi((double)k / (double)n, &sn, &cs);
            z[k] = fold_mode(F, L, n, k, double2{cs, sn});
        }
        __syncthreads();
        fft_forward<MAXN>(z, n, d.ring_rad + 16 * r);
        for (int j = threadIdx.x; j < n; j += kRingThreads) map[ring_pixel(d, r, j)] = w * z[j].x;
        return;
    }
    const int N = n >> 1;
    for (int k = threadIdx.x; 2 * k <= N; k += kRingThreads) {
        const int kp = k == 0 ? 0 : N - k;
        // p = exp(i pi k / n) gives every phase of the pair: at k + N it is i p,
        // at N - k i conj(p), at n - k -conj(p); w^k = conj(p)^2, w^(N-k) = -p^2
        double s, c;
        sincospi((double)k / (double)n, &s, &c);
        const double2 y0 = fold_mode(F, L, n, k, double2{c, s}), y1 = fold_mode(F, L, n, k + N, double2{-s, c});
        const double2 y2 = kp == k ? y0 : fold_mode(F, L, n, kp, double2{s, c});
        const double2 y3 = kp == k ? y1 : fold_mode(F, L, n, kp + N, double2{-c, s});
        const double c2 = c * c - s * s, s2 = 2.0 * c * s;
        const double2 a = double2{y0.x + y1.x, y0.y + y1.y}, ap = double2{y2.x + y3.x, y2.y + y3.y};
        const double2 b = cmul(double2{y0.x - y1.x, y0.y - y1.y}, double2{c2, -s2});
        const double2 bp = kp == k ? b : cmul(double2{y2.x - y3.x, y2.y - y3.y}, double2{-c2, -s2});
        // C_k = (a + conj ap) / 2 + i (b + conj bp) / 2, C_kp likewise with the roles swapped
        z[k] = double2{0.5 * (a.x + ap.x) - 0.5 * (b.y - bp.y), 0.5 * (a.y - ap.y) + 0.5 * (b.x + bp.x)};
        if (kp != k)
            z[kp] = double2{0.5 * (ap.x + a.x) - 0.5 * (bp.y - b.y), 0.5 * (ap.y - a.y) + 0.5 * (bp.x + b.x)};
    }
    __syncthreads();
    fft_forward<MAXN>(z, N, d.ring_rad + 16 * r);
    for (int j = threadIdx.x; j < N; j += kRingThreads) {
        map[ring_pixel(d, r, 2 * j)] = w * z[j].x;
        map[ring_pixel(d, r, 2 * j + 1)] = w * z[j].y;
    }
}

// The transpose: G_m^cos = c_m sum_j f_j cos(m phi_j), G_m^sin = sqrt(2)
// sum_j f_j sin(m phi_j) (c_0 = 1, c_m = sqrt(2)), from D = DFT_n(f) as
// exp(-i pi m / n) D_(m mod n).  Even n = 2N: Z = DFT_N(f_2r + i f_2r+1) gives
// D_q = E_q + w^q O_q with E_q = (Z_q + conj Z_N-q) / 2 and O_q = (Z_q - conj
// Z_N-q) / (2 i) (indices mod N).  With wmul the ring is first scaled by its
// pixel weight (the W of analysis).
template <int MAXN>
__global__ __launch_bounds__(kRingThreads) void k_ring_adj(ShtDesc d, const double *__restrict__ map,
                                                          double *__restrict__ gbuf, int wmul) {
    extern __shared__ double2 z[];
    const int r = ring_of_workgroup(d);
    if (r < 0) return;
    const int L = d.lmax, n = d.ring_n[r];
    const double w = wmul ? d.ring_w[r] : 1.0;
    const bool half = (n & 1) == 0;
    const int nf = half ? n >> 1 : n;
    if (half) {
        for (int j = threadIdx.x; j < nf; j += kRingThreads)
            z[j] = double2{w * map[ring_pixel(d, r, 2 * j)], w * map[ring_pixel(d, r, 2 * j + 1)]};
    } else {
        for (int j = threadIdx.x; j < n; j += kRingThreads) z[j] = double2{w * map[ring_pixel(d, r, j)], 0.0};
    }
    __syncthreads();
    fft_forward<MAXN>(z, nf, d.ring_rad + 16 * r);
    double *G = gbuf + (int64_t)r * (L + 1) * 2;
    for (int m = threadIdx.x; m <= L; m += kRingThreads) {
        const int q = m % n;
        double sn, cs;
        sincospi((double)m / (double)n, &sn, &cs);
        double2 v;
        if (half) {
            const int qq = q < nf ? q : q - nf, qp = qq == 0 ? 0 : nf - qq;
            const double2 zq = z[qq], zc = double2{z[qp].x, -z[qp].y};
            const double2 e = double2{0.5 * (zq.x + zc.x), 0.5 * (zq.y + zc.y)};
            const double2 o = double2{0.5 * (zq.y - zc.y), -0.5 * (zq.x - zc.x)};   // (zq - zc) / (2 i)
            // w^q = exp(-2 pi i m / n) = conj(exp(i pi m / n))^2
            const double2 wo = cmul(o, double2{cs * cs - sn * sn, -2.0 * cs * sn});
            v = double2{e.x + wo.x, e.y + wo.y};
        } else {
            v = z[q];
        }
        const double re = v.x * cs + v.y * sn;          // Re(exp(-i pi m / n) v)
        const double im = v.y * cs - v.x * sn;
        G[2 * m] = m == 0 ? re : kSqrt2 * re;
        G[2 * m + 1] = m == 0 ? 0.0 : -kSqrt2 * im;
    }
}

}  // namespace

// ring kernels for the plan's longest FFT length max_fft (<= kShtMaxRing)
template <typename F>
static void ring_dispatch(int max_fft, F &&f) {
    if (max_fft <= 1024) f(std::integral_constant<int, 1024>());
    else if (max_fft <= 2048) f(std::integral_constant<int, 2048>());
    else if (max_fft <= 4096) f(std::integral_constant<int, 4096>());
    else f(std::integral_constant<int, kShtMaxRing>());
}

// The attribute is set to the instantiation's own bound (MAXN complex values),
// not to this plan's longest FFT: plans of other sizes that use the same
// instantiation then never lower it below what one of them launches with.
hipError_t sht_prepare(int max_fft) {
    hipError_t e = hipSuccess;
    ring_dispatch(max_fft, [&](auto mx) {
        constexpr int M = decltype(mx)::value;
        const int bytes = M * (int)sizeof(double2);
        e = hipFuncSetAttribute((const void *)k_ring_syn<M>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_ring_adj<M>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    });
    return e;
}

hipError_t sht_synthesis(const ShtDesc &d, const double *alm, double *ac, double *as, double *fbuf, double *map,
                         bool weighted, hipStream_t st) {
    const int L = d.lmax;
    const int nt = (L + kMmTile) / kMmTile;
    if (alm)
        hipLaunchKernelGGL(k_alm_mm<true>, dim3(nt, nt), dim3(256), 0, st, alm, L, d.row_off, d.rec_k, ac, as,
                           nullptr);
    const dim3 grid(order_workgroups(L)), block(kLegThreads);
    auto syn = [&](auto r) {
        hipLaunchKernelGGL(k_leg_syn<decltype(r)::value>, grid, block, 0, st, d, d.row_off, d.rec_b, d.rec_k, ac,
                           as, fbuf);
    };
    // ring pairs per thread: the most rings (up to 6) whose passes leave at
    // most 1/16 of the threads idle, else one ring per thread
    const int nq = (d.nhalf + kLegThreads - 1) / kLegThreads;
    auto fits = [&](int r) { return 16L * d.nhalf >= 15L * ((nq + r - 1) / r) * r * kLegThreads; };
    if (fits(6)) syn(std::integral_constant<int, 6>());
    else if (fits(4)) syn(std::integral_constant<int, 4>());
    else if (fits(3)) syn(std::integral_constant<int, 3>());
    else if (fits(2)) syn(std::integral_constant<int, 2>());
    else syn(std::integral_constant<int, 1>());
    const size_t lds_ring = (size_t)d.max_fft * sizeof(double2);
    ring_dispatch(d.max_fft, [&](auto mx) {
        hipLaunchKernelGGL(k_ring_syn<decltype(mx)::value>, dim3(ring_workgroups(d)), dim3(kRingThreads), lds_ring, st, d, fbuf,
                           map, weighted ? 1 : 0);
    });
    return hipGetLastError();
}

hipError_t sht_adjoint(const ShtDesc &d, const double *map, double *gbuf, double *ac, double *as, double *alm,
                       bool weighted, hipStream_t st) {
    const int L = d.lmax;
    if (d.nhalf > kShtMaxHalfRings) return hipErrorInvalidValue;
    const size_t lds_ring = (size_t)d.max_fft * sizeof(double2);
    ring_dispatch(d.max_fft, [&](auto mx) {
        hipLaunchKernelGGL(k_ring_adj<decltype(mx)::value>, dim3(ring_workgroups(d)), dim3(kRingThreads), lds_ring, st, d, map,
                           gbuf, weighted ? 1 : 0);
    });
    // every ring pair in one pass: 128 threads with up to 8 ring pairs each
    // (half the partial sums of 256 threads), else 256 threads with 6 or 8
    auto adj = [&](auto t, auto r) {
        constexpr int T = decltype(t)::value, R = decltype(r)::value;
        hipLaunchKernelGGL((k_leg_adj<T, R>), dim3(order_workgroups(L)), dim3(T), 0, st, d, d.row_off, d.rec_b, d.rec_k, gbuf, ac,
                           as);
    };
    using T128 = std::integral_constant<int, 128>;
    using T256 = std::integral_constant<int, 256>;
    const int nq = (d.nhalf + 127) / 128;
    if (nq <= 1) adj(T128(), std::integral_constant<int, 1>());
    else if (nq == 2) adj(T128(), std::integral_constant<int, 2>());
    else if (nq == 3) adj(T128(), std::integral_constant<int, 3>());
    else if (nq == 4) adj(T128(), std::integral_constant<int, 4>());
    else if (nq <= 6) adj(T128(), std::integral_constant<int, 6>());
    else if (nq <= 8) adj(T128(), std::integral_constant<int, 8>());
    else if (nq <= 12) adj(T256(), std::integral_constant<int, 6>());
    else adj(T256(), std::integral_constant<int, 8>());
    const int nt = (L + kMmTile) / kMmTile;
    if (alm)
        hipLaunchKernelGGL(k_alm_mm<false>, dim3(nt, nt), dim3(256), 0, st, nullptr, L, d.row_off, d.rec_k, ac,
                           as, alm);
    return hipGetLastError();
}

}  // namespace sympix
