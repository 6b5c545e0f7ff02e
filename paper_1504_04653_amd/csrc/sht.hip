// Spherical harmonic transforms on the SymPix geometry (gfx950): synthesis
// f = Y a, its transpose Y^T f, the quadrature analysis Y^T W f of Eq. 1 and,
// built from them, the degrade theta_2 = W_2 Y_2 Y_obs^T theta of Eq. 14.
//
// Real orthonormal harmonics without the Condon-Shortley phase: Y_{l,0} =
// lambda_l0, Y_{l,+-m} = sqrt(2) lambda_lm cos / sin(m phi).  A transform
// splits into a Legendre part per m (over all rings, O(L^2 N_ring)) and a
// Fourier part per ring (O(n log n)):
//
//   k_leg_syn  one workgroup per m: F_m(ring) = sum_l a_lm lambda_lm(theta),
//              north and south rings of a pair together (lambda_lm(pi - t) =
//              (-1)^(l-m) lambda_lm(t): even and odd l - m summed apart)
//   k_ring_syn one workgroup per ring: the modes folded onto the ring's n
//              frequencies, an FFT in LDS, the ring scattered to SymPix order
//   k_ring_adj the transpose: gather, FFT, unfold to the modes m <= L
//   k_leg_adj  one workgroup per m: a_lm = sum_rings lambda_lm G_m(ring),
//              reduced across the workgroup eight degrees at a time
//
// lambda_lm is carried by the three-term recurrence in l from lambda_mm
// (tabulated on the host), on values scaled by a power of two that changes by
// 2^300 when they grow past 2^300, so that the far-below-range values near the
// poles at high m still reach the degrees where they matter.
#include <hip/hip_runtime.h>

#include "sht.hpp"

namespace sympix {
namespace {

constexpr int kShtThreads = 512;
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kBig = 0x1p300, kSmall = 0x1p-300;

__device__ __forceinline__ int64_t mm_off(int L, int m) {     // m-major layout: rows l = m..L
    return (int64_t)m * (L + 1) - (int64_t)m * (m - 1) / 2;
}

// ---------------------------------------------------------------------------
// Coefficient layout: (L+1)^2 entries at l^2 + l + m  <->  m-major rows of
// cos (m >= 0) and sin (m >= 1; the m = 0 row is zero) coefficients.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lm_of(int64_t idx, int &l, int &m) {
    int q = (int)sqrt((double)idx);
    while ((int64_t)q * q > idx) --q;
    while ((int64_t)(q + 1) * (q + 1) <= idx) ++q;
    l = q;
    m = (int)(idx - (int64_t)q * q - q);
}

__global__ __launch_bounds__(256) void k_alm_to_mm(const double *__restrict__ alm, int L,
                                                   double *__restrict__ ac, double *__restrict__ as) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)(L + 1) * (L + 1)) return;
    int l, m;
    lm_of(idx, l, m);
    if (m >= 0) {
        ac[mm_off(L, m) + l - m] = alm[idx];
        if (m == 0) as[mm_off(L, 0) + l] = 0.0;
    } else {
        as[mm_off(L, -m) + l + m] = alm[idx];
    }
}

__global__ __launch_bounds__(256) void k_mm_to_alm(const double *__restrict__ ac, const double *__restrict__ as,
                                                   int L, double *__restrict__ alm) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)(L + 1) * (L + 1)) return;
    int l, m;
    lm_of(idx, l, m);
    alm[idx] = m >= 0 ? ac[mm_off(L, m) + l - m] : as[mm_off(L, -m) + l + m];
}

// recurrence factors of degree l (l > m): lambda_l = alpha cos(t) lambda_{l-1}
// - gamma lambda_{l-2}; gamma = 0 at l = m + 1
__device__ __forceinline__ void rec_factors(int l, int m, double &alpha, double &gamma) {
    const double dl = l, dm = m;
    if (l == m + 1) {
        alpha = sqrt(2.0 * dm + 3.0);
        gamma = 0.0;
        return;
    }
    alpha = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
    const double beta = sqrt(((dl - 1.0) * (dl - 1.0) - dm * dm) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
    gamma = alpha * beta;
}

// ---------------------------------------------------------------------------
// Legendre synthesis.  Workgroup m; thread t takes the ring pairs t + 512 q
// (R of them at a time, interleaved for latency).  LDS: (alpha, gamma) and
// (a_cos, a_sin) per degree of this m, padded by kLegPad entries so that the
// loop reads ahead without a bound check.  Degrees go in pairs (odd i = l -
// m, then even), so that the parity of each is fixed; the test for the 2^300
// rescale is made once per pair (two steps of the recurrence grow a value by
// far less than the 2^723 left to the top of the double range).
// ---------------------------------------------------------------------------
constexpr int kLegPad = 8;

__device__ __forceinline__ void leg_fill(int m, int L, int nl, const double *ac, const double *as, double2 *sF,
                                         double2 *sA) {
    const int64_t off = mm_off(L, m);
    for (int i = threadIdx.x; i < nl + kLegPad; i += kShtThreads) {
        double al = 0.0, ga = 0.0;
        if (i > 0 && i < nl) rec_factors(m + i, m, al, ga);
        sF[i] = double2{al, ga};
        if (sA) sA[i] = i < nl ? double2{ac[off + i], as[off + i]} : double2{0.0, 0.0};
    }
}

template <int R>
__global__ __launch_bounds__(kShtThreads) void k_leg_syn(ShtDesc d, const double *__restrict__ ac,
                                                         const double *__restrict__ as, double *__restrict__ fbuf) {
    extern __shared__ double2 sh[];
    const int m = blockIdx.x, L = d.lmax, nl = L - m + 1;
    double2 *sF = sh, *sA = sh + nl + kLegPad;        // (alpha, gamma), (a_cos, a_sin)
    leg_fill(m, L, nl, ac, as, sF, sA);
    __syncthreads();
    for (int rp0 = threadIdx.x; rp0 < d.nhalf; rp0 += kShtThreads * R) {
        double ct[R], x[R], xp[R], ec[R], es[R], oc[R], os[R];
        int e[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int rp = min(rp0 + kShtThreads * q, d.nhalf - 1);
            ct[q] = d.ring_cos[rp];
            x[q] = d.lmm_mant[(int64_t)m * d.nhalf + rp];
            e[q] = d.lmm_exp[(int64_t)m * d.nhalf + rp];
            xp[q] = 0.0;
            ec[q] = sA[0].x * x[q];
            es[q] = sA[0].y * x[q];
            oc[q] = os[q] = 0.0;
        }
        double2 f1 = sF[1], a1 = sA[1], f2 = sF[2], a2 = sA[2];
        for (int i = 1; i < nl; i += 2) {
            const double2 g1 = sF[i + 2], b1 = sA[i + 2], g2 = sF[i + 3], b2 = sA[i + 3];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double x1 = fma(f1.x * ct[q], x[q], -f1.y * xp[q]);      // odd degree
                oc[q] = fma(a1.x, x1, oc[q]);
                os[q] = fma(a1.y, x1, os[q]);
                const double x2 = fma(f2.x * ct[q], x1, -f2.y * x[q]);       // even degree (zero past L)
                ec[q] = fma(a2.x, x2, ec[q]);
                es[q] = fma(a2.y, x2, es[q]);
                xp[q] = x1;
                x[q] = x2;
                if (fabs(x2) > kBig) {                // rescale the recurrence and its sums
                    x[q] *= kSmall;
                    xp[q] *= kSmall;
                    ec[q] *= kSmall;
                    es[q] *= kSmall;
                    oc[q] *= kSmall;
                    os[q] *= kSmall;
                    e[q] += 300;
                }
            }
            f1 = g1;
            a1 = b1;
            f2 = g2;
            a2 = b2;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int rp = rp0 + kShtThreads * q;
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
// Legendre transpose.  Workgroup m; thread t carries ring pairs t + 512 q (q <
// R) and adds lambda_lm (G(north) +- G(south)) over them, eight degrees at a
// time (four pairs, parities fixed as above); the workgroup then sums the
// 512 partials of each of the 16 values (cos, sin x 8 degrees) through LDS
// (row w read by 32 threads at consecutive addresses) and wave shuffles.
// Degrees past L read zero factors and are not written.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(kShtThreads) void k_leg_adj(ShtDesc d, const double *__restrict__ gbuf,
                                                         double *__restrict__ ac, double *__restrict__ as) {
    constexpr int CH = 8;
    extern __shared__ double2 sh[];
    const int m = blockIdx.x, L = d.lmax, nl = L - m + 1;
    const int nch = (nl + CH - 1) / CH;
    double2 *sF = sh;                                  // (alpha, gamma) per degree, zero past L
    double *sRed = (double *)(sh + nl + kLegPad);      // [2 CH][512]
    leg_fill(m, L, nl, nullptr, nullptr, sF, nullptr);  // nch CH <= nl + 7 < nl + kLegPad
    const int64_t off = mm_off(L, m);
    double ct[R], x[R], xp[R], fsc[R], pc[R], mc[R], ps[R], ms[R];
    int e[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int rp = threadIdx.x + kShtThreads * q;
        const bool ok = rp < d.nhalf;
        const int r = ok ? rp : 0;
        const int rs = d.nrings - 1 - r;
        ct[q] = d.ring_cos[r];
        x[q] = ok ? d.lmm_mant[(int64_t)m * d.nhalf + r] : 0.0;
        e[q] = d.lmm_exp[(int64_t)m * d.nhalf + r];
        fsc[q] = ldexp(1.0, e[q]);
        xp[q] = 0.0;
        const double *gn = gbuf + ((int64_t)r * (L + 1) + m) * 2;
        const double *gs = gbuf + ((int64_t)rs * (L + 1) + m) * 2;
        pc[q] = gn[0] + gs[0];
        mc[q] = gn[0] - gs[0];
        ps[q] = gn[1] + gs[1];
        ms[q] = gn[1] - gs[1];
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int i0 = c * CH;
        double vc[CH], vs[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) vc[j] = vs[j] = 0.0;
#pragma unroll
        for (int j = 0; j < CH; j += 2) {
            // degrees i0 + j (even i) and i0 + j + 1 (odd); i = 0 is lambda_mm itself
            const double2 f0 = sF[i0 + j], f1 = sF[i0 + j + 1];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                double x0 = x[q];
                if (i0 + j > 0) x0 = fma(f0.x * ct[q], x[q], -f0.y * xp[q]);
                const double x1 = fma(f1.x * ct[q], x0, -f1.y * x[q]);
                const double v0 = x0 * fsc[q], v1 = x1 * fsc[q];
                vc[j] = fma(v0, pc[q], vc[j]);
                vs[j] = fma(v0, ps[q], vs[j]);
                vc[j + 1] = fma(v1, mc[q], vc[j + 1]);
                vs[j + 1] = fma(v1, ms[q], vs[j + 1]);
                // carry (x0, x1) as (x_{i-1}, x_i) of the next pair: the next
                // even degree needs x_{i0+j+1} and x_{i0+j}
                xp[q] = x0;
                x[q] = x1;
                if (fabs(x1) > kBig) {
                    x[q] *= kSmall;
                    xp[q] *= kSmall;
                    e[q] += 300;
                    fsc[q] = ldexp(1.0, e[q]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            sRed[j * kShtThreads + threadIdx.x] = vc[j];
            sRed[(CH + j) * kShtThreads + threadIdx.x] = vs[j];
        }
        __syncthreads();
        const int row = threadIdx.x >> 5, seg = threadIdx.x & 31;
        double sum = 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) sum += sRed[row * kShtThreads + t * 32 + seg];   // 32 threads: 32 banks
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (seg == 0) {
            const int i = i0 + (row & (CH - 1));
            if (i < nl) {
                if (row < CH) ac[off + i] = sum;
                else as[off + i] = m == 0 ? 0.0 : sum;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// FFT in LDS: forward DFT z_q <- sum_j z_j exp(-2 pi i j q / n) for n =
// 2^a 3^b 5^c <= kShtMaxRing, by self-sorting (Stockham) passes of radix 2,
// 3, 4 and 5.  Pass with radix R over sub-transforms of length Ns: butterfly
// j takes z[j + r n/R] (r < R), twiddles them by exp(-2 pi i (j mod Ns) r /
// (Ns R)), applies the R-point DFT and writes output r to (j / Ns) Ns R +
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

template <int R>
__device__ __forceinline__ void fft_pass(double2 *z, int n, int Ns) {
    constexpr int MB = (kShtMaxRing / R + kShtThreads - 1) / kShtThreads;
    const int nb = n / R;
    double2 out[MB][R];
    int dst[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int j = threadIdx.x + kShtThreads * b;
        dst[b] = -1;
        if (j < nb) {
            const int k = j % Ns;
            double2 v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = z[j + r * nb];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                double sn, cs;
                sincospi(-2.0 * (double)(k * r) / (double)(Ns * R), &sn, &cs);
                v[r] = cmul(v[r], double2{cs, sn});
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

__device__ void fft_forward(double2 *z, int n, const int8_t *rad) {
    int Ns = 1;
    const int np = rad[0];
    for (int p = 1; p <= np; ++p) {
        const int R = rad[p];
        if (R == 4) fft_pass<4>(z, n, Ns);
        else if (R == 2) fft_pass<2>(z, n, Ns);
        else if (R == 3) fft_pass<3>(z, n, Ns);
        else fft_pass<5>(z, n, Ns);
        Ns *= R;
    }
}

// pixel of ring position j: tile j / k of the band, column j % k, this ring's
// row (folded into pix0)
__device__ __forceinline__ int64_t ring_pixel(const ShtDesc &d, int r, int j) {
    return d.ring_pix0[r] + (int64_t)(j / d.k) * d.k * d.k + (int64_t)(j % d.k) * d.k;
}

// f_j = Re sum_m H_m exp(i m phi_j), phi_j = 2 pi (j + 1/2) / n, with H_0 =
// F_0 and H_m = sqrt(2) (F_m^cos - i F_m^sin): fold m onto k = m mod n with the
// half-pixel phase exp(i pi m / n), then f = Re DFT(conj Z).  With wmul the
// ring is scaled by its pixel weight (W_2 of Eq. 14).
__global__ __launch_bounds__(kShtThreads) void k_ring_syn(ShtDesc d, const double *__restrict__ fbuf,
                                                          double *__restrict__ map, int wmul) {
    extern __shared__ double2 z[];
    const int r = blockIdx.x, L = d.lmax, n = d.ring_n[r];
    const double *F = fbuf + (int64_t)r * (L + 1) * 2;
    for (int k = threadIdx.x; k < n; k += kShtThreads) {
        double zr = 0.0, zi = 0.0;
        for (int m = k; m <= L; m += n) {
            const double hc = m == 0 ? F[0] : kSqrt2 * F[2 * m];
            const double hs = m == 0 ? 0.0 : -kSqrt2 * F[2 * m + 1];
            double sn, cs;
            sincospi((double)m / (double)n, &sn, &cs);
            zr += hc * cs - hs * sn;
            zi += hc * sn + hs * cs;
        }
        z[k] = double2{zr, -zi};
    }
    __syncthreads();
    fft_forward(z, n, d.ring_rad + 16 * r);
    const double w = wmul ? d.ring_w[r] : 1.0;
    for (int j = threadIdx.x; j < n; j += kShtThreads) map[ring_pixel(d, r, j)] = w * z[j].x;
}

// The transpose: G_m^cos = c_m sum_j f_j cos(m phi_j), G_m^sin = sqrt(2)
// sum_j f_j sin(m phi_j) (c_0 = 1, c_m = sqrt(2)), from D = DFT(f) as
// exp(-i pi m / n) D_(m mod n).  With wmul the ring is first scaled by its
// pixel weight (the W of analysis).
__global__ __launch_bounds__(kShtThreads) void k_ring_adj(ShtDesc d, const double *__restrict__ map,
                                                          double *__restrict__ gbuf, int wmul) {
    extern __shared__ double2 z[];
    const int r = blockIdx.x, L = d.lmax, n = d.ring_n[r];
    const double w = wmul ? d.ring_w[r] : 1.0;
    for (int j = threadIdx.x; j < n; j += kShtThreads) z[j] = double2{w * map[ring_pixel(d, r, j)], 0.0};
    __syncthreads();
    fft_forward(z, n, d.ring_rad + 16 * r);
    double *G = gbuf + (int64_t)r * (L + 1) * 2;
    for (int m = threadIdx.x; m <= L; m += kShtThreads) {
        const double2 v = z[m % n];
        double sn, cs;
        sincospi((double)m / (double)n, &sn, &cs);
        const double re = v.x * cs + v.y * sn;          // Re(exp(-i pi m / n) v)
        const double im = v.y * cs - v.x * sn;
        G[2 * m] = m == 0 ? re : kSqrt2 * re;
        G[2 * m + 1] = m == 0 ? 0.0 : -kSqrt2 * im;
    }
}

}  // namespace

hipError_t sht_prepare(int lmax, int max_ring) {
    const int leg_syn = 2 * (lmax + 1 + kLegPad) * (int)sizeof(double2);
    const int leg_adj = (lmax + 1 + kLegPad) * (int)sizeof(double2) + 16 * kShtThreads * (int)sizeof(double);
    const int ring = max_ring * (int)sizeof(double2);
    hipError_t e = hipSuccess;
    auto set = [&](const void *f, int bytes) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    };
    set((const void *)k_leg_syn<1>, leg_syn);
    set((const void *)k_leg_syn<2>, leg_syn);
    set((const void *)k_leg_syn<3>, leg_syn);
    set((const void *)k_leg_adj<1>, leg_adj);
    set((const void *)k_leg_adj<2>, leg_adj);
    set((const void *)k_leg_adj<3>, leg_adj);
    set((const void *)k_ring_syn, ring);
    set((const void *)k_ring_adj, ring);
    return e;
}

hipError_t sht_synthesis(const ShtDesc &d, const double *alm, double *ac, double *as, double *fbuf, double *map,
                         bool weighted, hipStream_t st) {
    const int L = d.lmax;
    const int64_t nalm = (int64_t)(L + 1) * (L + 1);
    if (alm) hipLaunchKernelGGL(k_alm_to_mm, dim3((unsigned)((nalm + 255) / 256)), dim3(256), 0, st, alm, L, ac, as);
    const size_t lds_leg = (size_t)2 * (L + 1 + kLegPad) * sizeof(double2);
    if (d.nhalf > 2 * kShtThreads)
        hipLaunchKernelGGL(k_leg_syn<3>, dim3(L + 1), dim3(kShtThreads), lds_leg, st, d, ac, as, fbuf);
    else if (d.nhalf > kShtThreads)
        hipLaunchKernelGGL(k_leg_syn<2>, dim3(L + 1), dim3(kShtThreads), lds_leg, st, d, ac, as, fbuf);
    else
        hipLaunchKernelGGL(k_leg_syn<1>, dim3(L + 1), dim3(kShtThreads), lds_leg, st, d, ac, as, fbuf);
    const size_t lds_ring = (size_t)d.max_ring * sizeof(double2);
    hipLaunchKernelGGL(k_ring_syn, dim3(d.nrings), dim3(kShtThreads), lds_ring, st, d, fbuf, map, weighted ? 1 : 0);
    return hipGetLastError();
}

hipError_t sht_adjoint(const ShtDesc &d, const double *map, double *gbuf, double *ac, double *as, double *alm,
                       bool weighted, hipStream_t st) {
    const int L = d.lmax;
    const size_t lds_ring = (size_t)d.max_ring * sizeof(double2);
    hipLaunchKernelGGL(k_ring_adj, dim3(d.nrings), dim3(kShtThreads), lds_ring, st, d, map, gbuf, weighted ? 1 : 0);
    const size_t lds_leg = (size_t)(L + 1 + kLegPad) * sizeof(double2) + (size_t)16 * kShtThreads * sizeof(double);
    if (d.nhalf > 2 * kShtThreads)
        hipLaunchKernelGGL(k_leg_adj<3>, dim3(L + 1), dim3(kShtThreads), lds_leg, st, d, gbuf, ac, as);
    else if (d.nhalf > kShtThreads)
        hipLaunchKernelGGL(k_leg_adj<2>, dim3(L + 1), dim3(kShtThreads), lds_leg, st, d, gbuf, ac, as);
    else
        hipLaunchKernelGGL(k_leg_adj<1>, dim3(L + 1), dim3(kShtThreads), lds_leg, st, d, gbuf, ac, as);
    const int64_t nalm = (int64_t)(L + 1) * (L + 1);
    if (alm) hipLaunchKernelGGL(k_mm_to_alm, dim3((unsigned)((nalm + 255) / 256)), dim3(256), 0, st, ac, as, L, alm);
    return hipGetLastError();
}

}  // namespace sympix
