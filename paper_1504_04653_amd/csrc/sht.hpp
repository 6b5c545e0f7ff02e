// Spherical harmonic transforms on the SymPix geometry: device tables of a
// transform plan and the launch functions (sht.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sympix {

constexpr int kShtMaxRing = 8192;   // longest ring the LDS FFT holds (complex FP64)
constexpr int kShtMaxL = 4095;      // largest band limit
constexpr int kShtMaxHalfRings = 2048;   // northern rings the Legendre transpose holds (8 per thread)
constexpr int kShtRowPad = 16;      // zero entries after each m-major row (read-ahead of the kernels)

// Device tables of one plan (grid, band limit L).  Rings j = 0 .. nrings-1
// from the north pole; ring nrings-1-j mirrors ring j, so the Legendre part
// runs over the nhalf = nrings/2 northern rings.
struct ShtDesc {
    int32_t lmax, nrings, nhalf, k, max_ring, max_fft;   // max_fft: longest ring FFT (n / 2 for even n, else n)
    const double *ring_cos;     // [nhalf] cos(theta) of the northern rings
    const double *lmm_mant;     // [L+1][nhalf] lambda_mm = mant * 2^exp
    const int32_t *lmm_exp;     // [L+1][nhalf]
    const int32_t *ring_n;      // [nrings] pixels on the ring
    const int64_t *ring_pix0;   // [nrings] pixel of ring position 0 (ring position j:
                                // + (j / k) k^2 + (j % k) k)
    const double *ring_w;       // [nrings] quadrature weight of each of the ring's pixels
    const int8_t *ring_rad;     // [nrings][16] passes of the ring's FFT (length n / 2 for even n, else n):
                                // count, then radices
    // m-major rows (row m: entries i = l - m = 0 .. L - m, then at least
    // kShtRowPad zeros; every row starts at a multiple of 4 entries)
    const int64_t *row_off;     // [L+1] first entry of row m
    const double *rec_b;        // b_i of the monic recurrence (b_0 = -1)
    const double *rec_k;        // K_i: the normalised factors' product over i's 64-degree chunk
};

// map = Y a (alm in the l^2 + l + m layout; nullptr: the m-major ac / as,
// held times K, are already filled); with weighted, map = W Y a.  fbuf: nrings (L+1) 2 doubles.
hipError_t sht_synthesis(const ShtDesc &d, const double *alm, double *ac, double *as, double *fbuf, double *map,
                         bool weighted, hipStream_t st);
// alm = Y^T map (weighted: Y^T W map); alm == nullptr leaves the result in the
// m-major ac / as (times K).  gbuf: nrings (L+1) 2 doubles.
hipError_t sht_adjoint(const ShtDesc &d, const double *map, double *gbuf, double *ac, double *as, double *alm,
                       bool weighted, hipStream_t st);
// Allow the ring kernels (the instantiation for FFTs up to max_fft) their
// largest LDS.
hipError_t sht_prepare(int max_fft);

}  // namespace sympix
