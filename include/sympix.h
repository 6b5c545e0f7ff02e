/*
 * sympix.h -- C ABI of the SymPix local-operator sampling library (gfx950).
 *
 * What it computes (Seljebotn & Eriksen, "SymPix: A spherical grid for
 * efficient sampling of rotationally invariant operators"):
 *   - the SymPix grid for a band limit lmax and tile size k (Section 2, Fig. 3);
 *   - the kernel b(x) = sum_l (2l+1)/(4 pi) b_l P_l(x) of a rotationally
 *     invariant operator with transfer function b_l (Eq. 10);
 *   - the local part of D-hat = Y D Y^T and B-hat = Y B Y^T (Eq. 16): elements
 *     between pixels in the same or in neighbouring tiles (Section 4.2);
 *   - the matching blocks of B-hat^T N^-1 B-hat for a diagonal pixel-space N^-1
 *     (Eq. 15), also on the two-hop pattern and with N^-1 on a second grid
 *     (Eq. 13);
 *   - the pixel-domain convolution B-hat f (Section 4.1);
 *   - spherical harmonic synthesis, its transpose, analysis (Eq. 1) and the
 *     N^-1 degrade of Eq. 14 on the SymPix geometry;
 *   - the block-Jacobi factor of D-hat + B-hat^T N^-1 B-hat and its solve
 *     (Section 4.2's system matrix).
 *
 * Conventions shared by every call
 * --------------------------------
 * Status: every call returns a sympix_status; on failure a thread-local
 *   message is available from sympix_last_error().  No C++ exception crosses
 *   this boundary.  Argument checks are synchronous.  Device work is queued on
 *   the caller's stream (a hipStream_t passed as void*, NULL = default stream)
 *   and is asynchronous: a device fault surfaces as SYMPIX_EHIP on a later
 *   call, or on the call itself when the environment variable SYMPIX_SYNC=1.
 * Ownership: the caller owns every buffer it passes.  "host" buffers are
 *   ordinary host memory of the stated length; "device" buffers are device
 *   pointers on the current HIP device.  The library owns the opaque handles
 *   and the device tables behind them; handles are immutable once created, so
 *   concurrent sample calls on different streams are safe.
 * Pixel layout (Section 2.4): bands in the order N0, S0, N1, S1, ...; inside a
 *   band tiles by increasing phi; inside a tile the ring index r (rings by
 *   increasing theta) runs fastest, then the column c.  Pixel index =
 *   tile * k^2 + c*k + r, so tile J owns pixels [J k^2, (J+1) k^2).
 * Block layout: a block (J, K) is k^2 x k^2 float64, row-major, row a = local
 *   pixel c*k + r of tile J, column b = local pixel of tile K.  Stored blocks
 *   are the pairs with K a neighbour of J and K >= J, ordered by J then K (the
 *   CSR of sympix_grid_blocks); lower blocks are the transposes.
 */
#ifndef SYMPIX_H
#define SYMPIX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SYMPIX_OK = 0,
    SYMPIX_EINVAL = -1,      /* bad argument: NULL handle/pointer, lmax < 1, k < 1, ... */
    SYMPIX_EINFEASIBLE = -2, /* the tile-count programme of Fig. 3 has no solution */
    SYMPIX_ENOMEM = -3,      /* host or device allocation failed */
    SYMPIX_EHIP = -4,        /* a HIP runtime call or kernel launch failed */
    SYMPIX_ESIZE = -5,       /* an output or input length does not match the grid */
    SYMPIX_EUNSUPPORTED = -6 /* valid request this library does not implement (see message) */
} sympix_status;

typedef enum {
    SYMPIX_FP64 = 0,   /* FP64 MFMA, FP64 accumulation */
    SYMPIX_FP32 = 1,   /* FP32 MFMA per term, FP64 accumulation across terms */
    SYMPIX_BF16X3 = 2, /* operands split in two BF16 parts, 3 products, FP32 MFMA accumulation
                          per term, FP64 across terms */
    SYMPIX_BF16X6 = 3  /* operands split in three BF16 parts, 6 products, otherwise as BF16X3 */
} sympix_precision;

typedef struct sympix_grid sympix_grid;     /* opaque, library-owned */
typedef struct sympix_kernel sympix_kernel; /* opaque, library-owned, bound to one grid */

typedef struct {
    int32_t lmax;            /* band limit given at creation */
    int32_t k;               /* tile size (k x k pixels per tile, k rings per band) */
    int32_t nrings;          /* lmax+1 rounded up to a multiple of 2k (Fig. 3) */
    int32_t nbands_hemi;     /* n = nrings / 2k bands per hemisphere */
    int64_t npix;            /* 2 k^2 sum_i T_i */
    int64_t ntiles;          /* npix / k^2 */
    int64_t nadjacency;      /* entries of the full tile adjacency (itself included) */
    int64_t nblocks;         /* stored blocks (J, K), K >= J */
    int64_t nterms;          /* sum over stored blocks of |nbr(J) & nbr(K)| */
    int64_t nunique;         /* distinct (band_I, band_J, phi offset) keys */
    double polar_margin;     /* right-hand side of Eq. 3 actually used */
    double y_pattern_max;    /* largest 1 - cos(gamma) between pixels of neighbouring tiles */
} sympix_dims;

/* Build the SymPix grid for (lmax, k): Gauss-Legendre rings (Section 2.1),
 * alpha_i from Eq. 3 at the pole-most ring of each band, tile counts from the
 * dynamic programme of Fig. 3 (band 1 may differ from band 0, as the caption
 * of Fig. 3 allows), the Section 2.4 layout, the neighbouring-tile relation and
 * the symmetry keys of Section 2.3.  Host only: no device is touched.
 *   polar_margin: right-hand side of Eq. 3; NaN selects the paper's
 *                 max(100, lmax/100).
 *   out:          receives the new handle (destroy with sympix_grid_destroy).
 * Errors: EINVAL (lmax < 1, k < 1, k > 64, lmax > 100000, out NULL),
 *         EINFEASIBLE (no tile layout), ENOMEM. */
sympix_status sympix_grid_create(int32_t lmax, int32_t k, double polar_margin, sympix_grid **out);

/* Free a grid and its device tables. NULL is ignored.  All kernels made from
 * the grid must be destroyed first and no call using it may be in flight. */
void sympix_grid_destroy(sympix_grid *g);

/* Sizes of the grid (host struct). Errors: EINVAL. */
sympix_status sympix_grid_dims(const sympix_grid *g, sympix_dims *out);

/* Ring tables, host buffers of length nrings, ring j counted from the north
 * pole: colatitude theta_j (zeros of P_nrings(cos theta)), Gauss-Legendre weight
 * w_j (Eq. 2), pixels on the ring n_j = k T, and the pixel index of the ring's
 * first pixel (phi = pi / n_j).  Any pointer may be NULL to skip it. */
sympix_status sympix_grid_rings(const sympix_grid *g, double *theta, double *weight,
                                int32_t *npix_ring, int64_t *first_pix);

/* Band tables in storage order (length 2 n): tiles T and alpha (Fig. 3), and
 * the index of the band's first (smallest-theta) ring.  NULL skips. */
sympix_status sympix_grid_bands(const sympix_grid *g, int32_t *tiles, int32_t *alpha,
                                int32_t *first_ring);

/* Colatitude theta and longitude phi of every pixel, in pixel order (host
 * buffers of npix values; either may be NULL).  Section 2.4 layout: pixel p of
 * a ring of n pixels sits at phi = 2 pi (p + 1/2) / n, the first one half a
 * pixel step from phi = 0 (Section 2.3), on the ring's Gauss-Legendre
 * colatitude (Section 2.1).  Errors: EINVAL (NULL grid). */
sympix_status sympix_grid_pixels(const sympix_grid *g, double *theta, double *phi);

/* Full tile adjacency as CSR: row_ptr[ntiles+1] (int64), col[nadjacency]
 * (int32, ascending, the tile itself included).  These are the "neighbouring
 * tiles" of Section 2.2 (the partner points a pixel needs lie in its own tile
 * and the tiles around it) and of the truncation in Section 4.2.  Same band:
 * t-1, t, t+1 mod T; neighbouring band (N_i-N_i+1, S_i-S_i+1, N_{n-1}-S_{n-1}):
 * closed phi intervals that meet; no neighbour across a pole.  Host buffers.
 * Errors: EINVAL (NULL grid). */
sympix_status sympix_grid_neighbours(const sympix_grid *g, int64_t *row_ptr, int32_t *col);

/* Stored blocks as CSR over J: row_ptr[ntiles+1], col[nblocks] = K >= J.
 * Section 4.2 keeps an element of D-hat or B-hat only when its two pixels lie
 * in the same or in neighbouring tiles, so the local part of either operator
 * is the blocks (J, K) with K in nbr(J); by symmetry the pairs K >= J are
 * stored and the rest are their transposes.  Host buffers, NULL skips.
 * Errors: EINVAL (NULL grid). */
sympix_status sympix_grid_blocks(const sympix_grid *g, int64_t *row_ptr, int32_t *col);

/* Stored-block patterns of B-hat^T N^-1 B-hat.  With B-hat local (Section
 * 4.2: zero unless the two pixels' tiles are the same or neighbours), block
 * (J, K) of the product is nonzero only where nbr(J) and nbr(K) meet.
 *   ONE_HOP: K in nbr(J), the pattern of D-hat (what sympix_sample_BtNB and
 *            sympix_sample_D_BtNB return);
 *   TWO_HOP: every (J, K) whose neighbourhoods meet, i.e. every nonzero block
 *            of the product. */
typedef enum { SYMPIX_PATTERN_ONE_HOP = 0, SYMPIX_PATTERN_TWO_HOP = 1 } sympix_pattern;

/* Blocks (J, K >= J) of a sympix_pattern as CSR over J: *nblocks, *nterms
 * (contraction terms over all its blocks), row_ptr[ntiles+1] (int64),
 * col[nblocks] (int32, ascending).  Host buffers, any may be NULL (query
 * *nblocks first to size col).  The two-hop pattern is built on the first
 * call that needs it.
 * Errors: EINVAL (NULL grid, unknown pattern), ENOMEM. */
sympix_status sympix_grid_pattern_blocks(const sympix_grid *g, int32_t pattern, int64_t *nblocks, int64_t *nterms,
                                         int64_t *row_ptr, int32_t *col);

/* Symmetry keys (Section 2.3): for every adjacency entry (I, J) in CSR order
 * its unique-block id uid[nadjacency]; and for every id its key
 * (band_I, band_J, delta = (t_J T_I - t_I T_J) mod T_I T_J), arrays of length
 * nunique.  A block B-hat_IJ depends on (I, J) only through this key.  NULL skips. */
sympix_status sympix_grid_unique(const sympix_grid *g, int32_t *uid, int32_t *key_band_i,
                                 int32_t *key_band_j, int64_t *key_delta);

/* Tabulate the kernel of Eq. 10 for transfer function coef_l[0..ncoef-1]
 * (host, ncoef = lmax + 1 of the grid; entries beyond are ignored, missing
 * ones are zero) and evaluate every unique local block of the grid with it.
 *   radius:  truncation radius in radians (pairs with gamma > radius give 0);
 *            <= 0 means no radial cut (only the tile pattern truncates).
 *   n_nodes: table size, >= 64 (65536 recommended; 0 selects 65536).  Nodes
 *            are uniform in s = sqrt(1 - cos gamma) over the pattern's range
 *            (or the radius, if smaller); lookups use 4-point Lagrange
 *            interpolation in s, mirrored at s = 0 where the kernel is even.
 *   stream:  hipStream_t for the device work.  The kernel's device tables are
 *            allocated in stream order on it and the coefficients are copied
 *            asynchronously, so the call does not wait for the device; work
 *            on other streams that uses the kernel must be ordered after it.
 * The FP64 recurrence in y = 1 - cos gamma runs on the device; the unique
 * blocks are stored in FP64 (row-major and transposed) and in FP32.
 * Errors: EINVAL, ESIZE (ncoef < 1), ENOMEM, EHIP. */
sympix_status sympix_kernel_tabulate(const sympix_grid *g, const double *coef_l, int32_t ncoef,
                                     double radius, int32_t n_nodes, void *stream,
                                     sympix_kernel **out);

/* Free a kernel. NULL is ignored.  The device memory is released in stream
 * order on the null stream (after the work already queued on blocking
 * streams); work on non-blocking streams that uses the kernel must have
 * completed. */
void sympix_kernel_destroy(sympix_kernel *kr);

/* Evaluate the tabulated kernel (with its radial cut) at n arguments
 * y = 1 - cos gamma (device buffers y_dev[n] in, out_dev[n] out).  For tests of
 * the interpolation; y beyond the table domain is clamped to its end. */
sympix_status sympix_kernel_eval(const sympix_kernel *kr, const double *y_dev, double *out_dev,
                                 int64_t n, void *stream);

/* Local blocks of D-hat (Eq. 16 with Section 4.2's truncation) for the kernel
 * d: out_dev (device, float64) receives nblocks * k^4 values in stored-block
 * order.  Called with the beam kernel it returns the local blocks of B-hat.
 * Errors: EINVAL (NULL, kernel of another grid), ESIZE (out_len !=
 * nblocks k^4), EUNSUPPORTED (k != 8), EHIP. */
sympix_status sympix_sample_D(const sympix_grid *g, const sympix_kernel *d, double *out_dev,
                              int64_t out_len, void *stream);

/* Pixel-domain convolution (Section 4.1): out_i = sum_j b(n_i . n_j) f_j over
 * the pairs whose tiles are the same or neighbouring (and within the kernel's
 * radius), i.e. out = B-hat f with the local blocks of kernel b; a plain sum
 * over samples, no quadrature weights.  f_dev and out_dev: device, float64,
 * npix values in pixel order, 16-byte aligned, not overlapping.  FP64
 * throughout, bitwise reproducible run to run.
 * Errors: EINVAL (NULL, overlap, misalignment, kernel of another grid), ESIZE
 * (f_len or out_len != npix), EUNSUPPORTED (k != 8), EHIP. */
sympix_status sympix_convolve(const sympix_grid *g, const sympix_kernel *b, const double *f_dev,
                              int64_t f_len, double *out_dev, int64_t out_len, void *stream);

/* Stored blocks of B-hat^T N^-1 B-hat (Eq. 15):
 *   C_JK = sum_{I in nbr(J) & nbr(K)} B_IJ^T diag(ninv_I) B_IK,
 * with ninv_dev (device, float64, npix values in pixel order, 32-byte aligned,
 * >= 0; negative or NaN values are not checked and give undefined results) and
 * out_dev (device, float64, nblocks k^4 values, stored-block order, 16-byte
 * aligned, not overlapping ninv_dev).
 *   prec: a sympix_precision.  FP64 is bitwise reproducible run to run.
 * Errors: EINVAL (NULL, misalignment, out_dev overlapping ninv_dev, kernel of
 *         another grid or device), ESIZE (ninv_len != npix or out_len !=
 *         nblocks k^4), EUNSUPPORTED (k != 8), EHIP. */
sympix_status sympix_sample_BtNB(const sympix_grid *g, const sympix_kernel *b, const double *ninv_dev,
                                 int64_t ninv_len, int32_t prec, double *out_dev, int64_t out_len,
                                 void *stream);

/* sympix_sample_BtNB without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same arguments, kernels and results
 * (bitwise equal to sympix_sample_BtNB in every mode); the N^-1 operand
 * scratch of the FP32 and split-BF16 modes is a static device array of the
 * library (96 MiB per device, held until the process ends) instead of a
 * stream-ordered allocation, and FP64 needs none.
 * Limits and rules:
 *   - FP32 / BF16X3 / BF16X6: npix <= 16777216 (2^24; lmax 3000 at k = 8 has
 *     13,038,976), else ESIZE.  FP64: any size.
 *   - The grid's device tables must already exist on the current device
 *     (they do once a kernel of this grid has been tabulated there).
 *   - Every allocation-free call on a device shares that device's array:
 *     calls whose launches overlap in time on one device race and give
 *     undefined results; order them on one stream (or with events).  The
 *     array keeps the last call's contents; each call rewrites the part it
 *     reads before reading it.
 * Errors: as sympix_sample_BtNB, plus ESIZE for a grid beyond the limit and
 * EINVAL when the grid's tables are not on the device. */
sympix_status sympix_sample_BtNB_noalloc(const sympix_grid *g, const sympix_kernel *b, const double *ninv_dev,
                                         int64_t ninv_len, int32_t prec, double *out_dev, int64_t out_len,
                                         void *stream);

/* B-hat^T N^-1 B-hat (Eq. 15) on the blocks of a sympix_pattern, in its
 * stored-block order; out_len = that pattern's nblocks k^4.  The two-hop
 * blocks (J, K) not in the one-hop pattern have the terms I in nbr(J) and
 * nbr(K), one to a few.  Otherwise as sympix_sample_BtNB, which is this call
 * with SYMPIX_PATTERN_ONE_HOP.
 * Errors: EINVAL (also an unknown pattern), ESIZE, ENOMEM, EUNSUPPORTED, EHIP. */
sympix_status sympix_sample_BtNB_pattern(const sympix_grid *g, const sympix_kernel *b, const double *ninv_dev,
                                         int64_t ninv_len, int32_t prec, int32_t pattern, double *out_dev,
                                         int64_t out_len, void *stream);

/* Both local operators of Eq. 16 in one call: outD_dev receives the D-hat
 * blocks of kernel d (as sympix_sample_D) and outC_dev the B-hat^T N^-1 B-hat
 * blocks of kernel b (as sympix_sample_BtNB with the same prec), bitwise equal
 * to the two separate calls.  One launch writes both: the D-hat copies, bound
 * by HBM writes, proceed under the contraction's arithmetic.  outD_dev and
 * outC_dev: device, float64, nblocks k^4 values
 * each, stored-block order, 16-byte aligned, not overlapping each other or
 * ninv_dev.  Both kernels must belong to g and live on the current device.
 * Errors: EINVAL (NULL, overlap, misalignment, kernel of another grid or
 * device), ESIZE (ninv_len != npix or an output length != nblocks k^4),
 * EUNSUPPORTED (k != 8), EHIP. */
sympix_status sympix_sample_D_BtNB(const sympix_grid *g, const sympix_kernel *d, const sympix_kernel *b,
                                   const double *ninv_dev, int64_t ninv_len, int32_t prec, double *outD_dev,
                                   int64_t outD_len, double *outC_dev, int64_t outC_len, void *stream);

/* ---- Block-Jacobi factor of the system matrix (Section 4.2) --------------------
 * Section 4.2 solves with the matrix D-hat + B-hat^T N^-1 B-hat, and the local
 * blocks exist to build preconditioners or smoothers for its iterative
 * solution.  These two calls build and apply the block-Jacobi one: per tile
 * J the diagonal block A_J = D_JJ + C_JJ, its Cholesky factor, and
 * x_J = A_J^-1 r_J.  Device kernels for k = 8. */

/* For every tile J: A_J = D_JJ + C_JJ from the stored blocks (J, J) of D_dev
 * (sympix_sample_D layout) and C_dev (sympix_sample_BtNB layout; NULL with
 * C_len 0 factors D_JJ alone), both device float64 of nblocks k^4 values.
 * Only the upper triangle of A_J is read.  U_dev (device float64, ntiles k^4
 * values, tile J's block at J k^4) receives the upper triangular U_J with
 * A_J = U_J^T U_J, row-major, zeros below the diagonal; info_dev (device
 * int32, ntiles values) receives 0, or j + 1 when the pivot of row j is not
 * positive (A_J is not numerically positive definite; U_J is then
 * unspecified).  Pivots are scaled by their reciprocal.  Buffers 16-byte
 * aligned (info 4-byte), outputs not overlapping any other buffer.
 * Errors: EINVAL (NULL, misalignment, overlap), ESIZE (lengths), EUNSUPPORTED
 * (k != 8), EHIP. */
sympix_status sympix_factor_diag(const sympix_grid *g, const double *D_dev, int64_t D_len, const double *C_dev,
                                 int64_t C_len, double *U_dev, int64_t U_len, int32_t *info_dev, int64_t info_len,
                                 void *stream);

/* x_J = A_J^-1 r_J = (U_J^T U_J)^-1 r_J for every tile J (forward then back
 * substitution), with U_dev from sympix_factor_diag (ntiles k^4 values) and
 * r_dev, x_dev device float64 of npix values in pixel order (tile J owns
 * pixels [J k^2, (J+1) k^2)).  x_dev may be r_dev itself (in place) but may
 * not overlap it otherwise, nor U_dev.  Tiles whose factor failed give
 * unspecified values.
 * Errors: EINVAL (NULL, misalignment, overlap), ESIZE (lengths), EUNSUPPORTED
 * (k != 8), EHIP. */
sympix_status sympix_solve_diag(const sympix_grid *g, const double *U_dev, int64_t U_len, const double *r_dev,
                                int64_t r_len, double *x_dev, int64_t x_len, void *stream);

/* ---- Two grids: B-hat = Y_2 B Y_1^T (Eqs. 13 and 16) --------------------------
 * Eq. 13 moves N^-1 onto an auxiliary SymPix grid Y_2, which may differ from
 * the grid Y_1 of the unknowns (Section 4.2: with Y_2 at twice the band limit
 * of Y_1 the substitution holds to about 1e-10); B-hat = Y_2 B Y_1^T then has
 * a row per pixel of Y_2 and a column per pixel of Y_1, and Eq. 15 asks for
 * B-hat^T N_2^-1 B-hat on the stored blocks of Y_1.  An element of B-hat is
 * b(n_i . n_j) with the Eq. 10 kernel summed over l <= min(lmax_1, lmax_2).
 * Section 4.2's truncation ("same or neighbouring tiles") needs a relation
 * between tiles of two grids, which the paper does not give; this library
 * places each tile of Y_2 in the tile of Y_1 that contains its centre
 * (centres and band ranges [ik/R, (i+1)k/R] pi as exact rationals, half-open
 * to the south and east) and pairs it with that tile's neighbours, so the
 * truncation reaches as far as on one grid.  With Y_2 = Y_1 every table, and
 * every result, is bitwise that of the one-grid calls.  Both grids must have
 * the same k (8 for device sampling); blocks are k^2 x k^2. */
typedef struct sympix_cross sympix_cross;   /* opaque, library-owned; refers to both grids */

typedef struct {
    int32_t lmax_eff;        /* min(lmax_1, lmax_2): band limit of the kernel series */
    int32_t max_terms;       /* largest number of contraction terms of one stored block */
    int64_t nadjacency;      /* blocks of B-hat kept: pairs (tile I of Y_2, tile J of Y_1) */
    int64_t nunique;         /* distinct (band of I, band of J, phi offset) keys */
    int64_t nblocks;         /* stored blocks of B-hat^T N_2^-1 B-hat (those of Y_1) */
    int64_t nterms;          /* sum over stored blocks of the tiles I of Y_2 they share */
    double y_pattern_max;    /* largest 1 - cos(gamma) over the kept pairs */
} sympix_cross_sizes;

/* Tables of the pair (g2 = Y_2 auxiliary, g1 = Y_1); host only.  Both grids
 * must outlive the pair.  Errors: EINVAL (NULL), EUNSUPPORTED (different k),
 * ENOMEM. */
sympix_status sympix_cross_create(const sympix_grid *g2, const sympix_grid *g1, sympix_cross **out);

/* Free a pair and its device tables.  NULL is ignored; its kernels must be
 * destroyed first. */
void sympix_cross_destroy(sympix_cross *x);

/* Sizes of the pair.  Errors: EINVAL. */
sympix_status sympix_cross_dims(const sympix_cross *x, sympix_cross_sizes *out);

/* The tile relation (host buffers, NULL skips): container[ntiles_2] = the tile
 * of Y_1 holding each tile's centre; CSR over the tiles I of Y_2,
 * row_ptr[ntiles_2 + 1], col[nadjacency] = tiles J of Y_1 (ascending), and
 * uid[nadjacency] = each block's unique id.  Errors: EINVAL. */
sympix_status sympix_cross_neighbours(const sympix_cross *x, int32_t *container, int64_t *row_ptr, int32_t *col,
                                      int32_t *uid);

/* Key of every unique block: (band of I in Y_2, band of J in Y_1,
 * delta = (t_J T_I - t_I T_J) mod T_I T_J), arrays of nunique.  NULL skips. */
sympix_status sympix_cross_unique(const sympix_cross *x, int32_t *key_band_i, int32_t *key_band_j,
                                  int64_t *key_delta);

/* sympix_kernel_tabulate for the pair: the Eq. 10 kernel of coef_l up to
 * lmax_eff, tabulated over the pair's pattern, and every unique block of
 * B-hat = Y_2 B Y_1^T.  The handle serves sympix_sample_B_cross,
 * sympix_sample_BtNB_cross, sympix_kernel_eval and sympix_kernel_destroy.
 * Arguments and errors as sympix_kernel_tabulate. */
sympix_status sympix_kernel_tabulate_cross(const sympix_cross *x, const double *coef_l, int32_t ncoef,
                                           double radius, int32_t n_nodes, void *stream, sympix_kernel **out);

/* The kept blocks of B-hat (Eq. 16 with the truncation above): out_dev
 * (device, float64, nadjacency k^4 values, 16-byte aligned) receives block
 * (I, J) for each relation entry in CSR order, row a = local pixel of I (on
 * Y_2), column b = local pixel of J (on Y_1), row-major.
 * Errors: EINVAL (NULL, kernel of another pair), ESIZE, EUNSUPPORTED (k != 8),
 * EHIP. */
sympix_status sympix_sample_B_cross(const sympix_cross *x, const sympix_kernel *b, double *out_dev, int64_t out_len,
                                    void *stream);

/* B-hat^T N_2^-1 B-hat (Eq. 15) on the stored blocks of Y_1:
 *   C_JK = sum_{I of Y_2 related to J and K} B_IJ^T diag(ninv2_I) B_IK,
 * ninv2_dev (device, float64, npix of Y_2 in its pixel order, 32-byte
 * aligned), out_dev (device, float64, nblocks k^4 in the stored-block order of
 * Y_1, 16-byte aligned, not overlapping ninv2_dev); prec any
 * sympix_precision, on the same kernels as sympix_sample_BtNB.
 * Errors: EINVAL (NULL, misalignment, overlap, kernel of another pair, unknown
 * prec), ESIZE (ninv2_len != npix of Y_2, out_len != nblocks k^4),
 * EUNSUPPORTED (k != 8, more than 128 terms in a block), ENOMEM, EHIP. */
sympix_status sympix_sample_BtNB_cross(const sympix_cross *x, const sympix_kernel *b, const double *ninv2_dev,
                                       int64_t ninv2_len, int32_t prec, double *out_dev, int64_t out_len,
                                       void *stream);

/* ---- Batches: many B-hat^T N^-1 B-hat problems in one graph launch ----------
 * Eq. 15 evaluated for n independent problems (own grid, beam kernel, N^-1 and
 * output each) by one captured HIP graph: a persistent contraction in FP64
 * MFMA, FP32 MFMA or split-BF16 MFMA (the latter two with FP64 accumulation
 * across contraction tiles, as the single-problem modes) pulls (problem,
 * 64-block tile) work items from per-XCD queues.  Results are bitwise
 * identical to sympix_sample_BtNB(..., prec, ...) per problem, under every
 * schedule and tile shape. */
typedef struct sympix_batch sympix_batch;

typedef struct {
    const sympix_grid *g;
    const sympix_kernel *b;   /* beam kernel tabulated for g */
    const double *ninv_dev;   /* device, float64, npix values, 8-byte aligned (32-byte for SYMPIX_FP64) */
    int64_t ninv_len;         /* must be npix */
    double *out_dev;          /* device, float64, nblocks k^4 values, 16-byte aligned */
    int64_t out_len;          /* must be nblocks k^4 */
} sympix_problem;

typedef enum {
    SYMPIX_SCHED_XCD_QUEUES = 0,  /* persistent; one queue per XCD, items in grid order (default) */
    SYMPIX_SCHED_GLOBAL_LPT = 1,  /* persistent; one queue, largest items first */
    SYMPIX_SCHED_PER_PROBLEM = 2, /* one class-GEMM launch per problem, in sequence */
    SYMPIX_NSCHED = 3
} sympix_schedule;

/* Tile shape of the work items: member tiles of 64 stored blocks (tails of
 * 32 / 16, the default), or of 32 (tails of 16), which wastes less work on
 * the small classes of low-lmax grids.  A plan is schedule + SYMPIX_NSCHED *
 * tiling. */
typedef enum {
    SYMPIX_TILES_64 = 0,
    SYMPIX_TILES_32 = 1,
    SYMPIX_NTILINGS = 2
} sympix_tiling;

/* Build a batch over problems p[0..n) (copied; the buffers they point to must
 * stay allocated, and the grids and kernels alive, until the batch is
 * destroyed) and capture its graph with the default schedule (or the plan the
 * tuner chose earlier in this process for the same problems and mode).  prec:
 * any sympix_precision.  The batch owns its device tables and its N^-1
 * operand scratch (none in FP64, which reads N^-1 directly; 4 npix bytes per
 * problem in FP32, 6 in the split-BF16 modes).  stream: the call synchronises
 * it once while uploading tables.
 * Errors: EINVAL (NULL, n < 1, misaligned or overlapping outputs, problems on
 * another device, unknown prec), ESIZE (a length mismatch), EUNSUPPORTED
 * (k != 8), ENOMEM, EHIP. */
sympix_status sympix_batch_create(const sympix_problem *p, int32_t n, int32_t prec, void *stream,
                                  sympix_batch **out);

/* Re-capture the batch's graph with schedule s (a sympix_schedule), keeping
 * its tile shape.  Re-capturing rewrites the batch's work-item tables, so the
 * call first waits on the host for the batch's last launch (on any stream) to
 * complete; a launch made on another thread while this call runs is not
 * allowed. */
sympix_status sympix_batch_set_schedule(sympix_batch *bt, int32_t s);

/* Re-capture the batch's graph with tile shape t (a sympix_tiling), keeping
 * its schedule.  Waits for the batch's last launch as
 * sympix_batch_set_schedule does. */
sympix_status sympix_batch_set_tiling(sympix_batch *bt, int32_t t);

/* Autotune: time one launch of every plan (schedule and tile shape) on stream
 * (after one warm-up launch each; the outputs are overwritten), keep the
 * fastest and report its plan in *chosen and the times in
 * ms_out[SYMPIX_NSCHED * SYMPIX_NTILINGS], indexed by plan (either may be
 * NULL).  The choice is remembered for batches of the same problems and mode
 * in this process and, when the environment variable SYMPIX_TUNE_CACHE names
 * a file, in that file (one "<shape>\t<plan>" line per batch shape, keyed by
 * the gfx architecture, HIP runtime version, mode and every problem's lmax
 * and block count), where sympix_batch_create of a later process finds it.
 * Each re-capture first waits for the batch's previous launch, so the call
 * may follow sympix_batch_launch on any stream.
 * Errors: EINVAL (NULL, the cache file cannot be written), EHIP. */
sympix_status sympix_batch_tune(sympix_batch *bt, void *stream, int32_t *chosen, double *ms_out);

/* The plan the batch's graph was captured with (schedule + SYMPIX_NSCHED *
 * tiling).  Errors: EINVAL (NULL). */
sympix_status sympix_batch_plan(const sympix_batch *bt, int32_t *plan);

/* Enqueue the batch's graph on stream: converts every N^-1 to the operand
 * format (FP32, or BF16 parts; FP64 reads it as given) and writes every
 * output.  Launches of one batch must not overlap in time (they share its
 * queue counters and scratch): launch it on one stream, or order the streams. */
sympix_status sympix_batch_launch(sympix_batch *bt, void *stream);

/* Free a batch. NULL is ignored.  No launch of it may be in flight. */
void sympix_batch_destroy(sympix_batch *bt);

/* ------------------------------------------------------------------------
 * Spherical harmonic transforms on the SymPix geometry (Section 2.1, Eq. 1)
 * and the N^-1 degrade of Eq. 14.
 *
 * Basis: real orthonormal harmonics without the Condon-Shortley phase,
 *   Y_{l,0} = lambda_l0(theta),  Y_{l,m} = sqrt(2) lambda_lm(theta) cos(m phi),
 *   Y_{l,-m} = sqrt(2) lambda_lm(theta) sin(m phi)  (0 < m <= l <= L),
 * lambda_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta), P_l^m >= 0
 * near the north pole, so that Y (npix x (L+1)^2) is a real matrix and Y^T its
 * transpose.  Coefficient vectors: float64, (L+1)^2 entries, entry l^2 + l + m
 * for the coefficient of Y_{l,m}.  Maps: float64, npix values in the grid's
 * pixel order (sympix_grid_pixels).  W: per pixel, the Gauss-Legendre weight
 * of its ring times 2 pi / n_ring (the quadrature rule of Eq. 1).  Every mode
 * m <= L is kept on every ring (no mode is dropped near the poles).
 * ------------------------------------------------------------------------ */
typedef struct sympix_sht sympix_sht;

/* Plan for the transforms of band limit lmax_sh on grid g, on the current
 * device: ring tables, lambda_mm per ring and m, the recurrence's per-degree
 * values and the plan's work buffers (about 16 nrings (L+1) + 32 (L+1)(L+2)/2
 * + 12 (nrings/2)(L+1) bytes).  The
 * grid must outlive the plan.  Calls that use one plan (the transforms below,
 * and a degrade naming it) share its work buffers and must not overlap in
 * time: issue them on one stream, or order the streams.
 * Errors: EINVAL (NULL, lmax_sh < 0), EUNSUPPORTED (lmax_sh > 4095, more
 * than 4096 rings, a ring longer than 8192 pixels or not of the form
 * 2^a 3^b 5^c), ENOMEM, EHIP. */
sympix_status sympix_sht_create(const sympix_grid *g, int32_t lmax_sh, sympix_sht **out);

/* Free a plan (after its last call has completed). NULL is ignored. */
void sympix_sht_destroy(sympix_sht *s);

/* Synthesis map = Y alm: alm_dev (device, (L+1)^2 values), map_dev (device,
 * npix values); both 8-byte aligned, not overlapping.
 * Errors: EINVAL (NULL, overlap, plan on another device), ESIZE (alm_len !=
 * (L+1)^2, map_len != npix), EHIP. */
sympix_status sympix_sht_synthesis(sympix_sht *s, const double *alm_dev, int64_t alm_len, double *map_dev,
                                   int64_t map_len, void *stream);

/* Transpose alm = Y^T map (no quadrature weights).  Arguments and errors as
 * sympix_sht_synthesis. */
sympix_status sympix_sht_adjoint(sympix_sht *s, const double *map_dev, int64_t map_len, double *alm_dev,
                                 int64_t alm_len, void *stream);

/* Analysis alm = Y^T W map (Eq. 1).  Arguments and errors as
 * sympix_sht_synthesis. */
sympix_status sympix_sht_analysis(sympix_sht *s, const double *map_dev, int64_t map_len, double *alm_dev,
                                  int64_t alm_len, void *stream);

/* The degrade of Eq. 14, theta_2 = W_2 Y_2 Y_obs^T theta_obs: theta_obs_dev on
 * the grid of obs (npix_obs values), theta2_dev on the grid of target (npix_2
 * values); Y_obs^T carries no ring weights, W_2 is the target grid's
 * quadrature weight.  Both plans must have the same band limit and device.
 * Errors: EINVAL (NULL, overlap, band limits or devices differ), ESIZE, EHIP. */
sympix_status sympix_sht_degrade(sympix_sht *obs, sympix_sht *target, const double *theta_obs_dev,
                                 int64_t obs_len, double *theta2_dev, int64_t target_len, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *sympix_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SYMPIX_H */
