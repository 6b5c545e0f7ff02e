// Host-side SymPix geometry: rings, tile counts, layout, tile adjacency,
// symmetry keys and the contraction term lists.  Pure C++17, no device code.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sympix {

// One contraction term of an output block (J, K): C_JK += B_IJ^T diag(w_I) B_IK.
constexpr int kConvTiles = 32;   // output tiles per convolution chunk

struct Term {
    int32_t uid_a;  // unique block of (I -> J)
    int32_t uid_b;  // unique block of (I -> K)
    int32_t tile;   // I (its N^-1 values are pixels [I k^2, (I+1) k^2))
    int32_t pad;
};

// Stored blocks whose contraction tiles carry the same multiset of
// (unique B_IJ, unique B_IK) pairs: C_m = sum_(e,p) w[I_e(m)*k^2 + p] * M_e[p][ab]
// with M_e[p][(a,b)] = B_IJ[p][a] B_IK[p][b] shared by every block m.
struct BlockClass {
    int32_t nterms, nblocks;
    int32_t term0;   // first (uid_a, uid_b) pair in class_terms (pairs)
    int32_t blk0;    // first block in class_blk
    int64_t itab0;   // first entry in class_itab (nblocks * nterms, block-major)
    int32_t sym;     // 1 if every term pairs a unique block with itself: the
                     // members' blocks are symmetric (C_m[a][b] = C_m[b][a])
    int32_t pad;
};

// The contraction of a stored-block pattern in class-GEMM form.
struct ClassTables {
    std::vector<BlockClass> classes;
    std::vector<int32_t> class_terms;   // 2 per term: uid_a, uid_b
    std::vector<int32_t> class_blk;     // stored-block index of each class member
    std::vector<int32_t> class_itab;    // tile I of each (member, term)
    std::vector<int32_t> mtiles;        // 4 per member tile: class, first member,
                                        // 16-row groups (1, 2 or 4), 0
    std::vector<int32_t> mtiles32;      // the same with tiles of at most 32 rows
                                        // (groups 1 or 2): a tile shape for batches
    std::vector<int32_t> gtiles;        // mtiles in the order of a one-workgroup-per-tile
    std::vector<int32_t> gtiles32;      // launch (slot 8 i + x: the i-th tile run on
                                        // XCD x; groups 0: an empty slot), and mtiles32
    int32_t max_class_terms = 0;
};

// A further stored-block pattern of B-hat^T N^-1 B-hat: blocks (J, K >= J) as
// CSR over J, their contraction terms (CSR, I ascending) and classes.
struct Pattern {
    std::vector<int64_t> blk_ptr;
    std::vector<int32_t> blk_col;
    std::vector<int64_t> term_ptr;
    std::vector<Term> terms;
    ClassTables cls;
    int64_t nblocks() const { return (int64_t)blk_col.size(); }
};

struct Geometry {
    int32_t lmax = 0, k = 0, nrings = 0, nbands_hemi = 0;
    double margin = 0.0;

    // rings, j = 0 at the north pole
    std::vector<double> theta, sin_theta, cos_theta, weight;
    std::vector<int32_t> ring_npix;
    std::vector<int64_t> ring_first_pix;

    // per northern band i (Fig. 3)
    std::vector<int32_t> alpha_north, tiles_north;

    // bands in storage order N0, S0, N1, S1, ...
    std::vector<int32_t> band_tiles, band_alpha, band_ring0;
    std::vector<int64_t> band_tile0;

    int64_t npix = 0, ntiles = 0;
    std::vector<int32_t> tile_band;   // band of every tile

    // full tile adjacency (CSR, itself included, ascending)
    std::vector<int64_t> adj_ptr;
    std::vector<int32_t> adj_col;
    std::vector<int32_t> adj_uid;     // unique-block id of each (I, J) entry

    // symmetry keys, one per unique block, and a representative tile pair
    std::vector<int32_t> key_band_i, key_band_j;
    std::vector<int64_t> key_delta;
    std::vector<int32_t> rep_i, rep_j;

    // stored blocks (J, K >= J) as CSR over J, and per block its D-hat uid
    std::vector<int64_t> blk_ptr;
    std::vector<int32_t> blk_col;
    std::vector<int32_t> blk_uid;

    // D-hat expansion: stored blocks ordered by unique block, and work items
    // of at most 64 of them, 4 ints each {uid, first in exp_blk, count, 0}
    std::vector<int32_t> exp_blk;
    std::vector<int32_t> exp_items;

    // contraction terms per stored block (CSR, I ascending)
    std::vector<int64_t> term_ptr;
    std::vector<Term> terms;

    // block classes for the GEMM form of the contraction, and its m-tiles
    ClassTables cls;

    // convolution g = B-hat f: chunks of up to kConvTiles consecutive output
    // tiles of one band {first tile, tiles, first slot, slots}; per slot a
    // unique block and, for each tile, the input tile K it multiplies (-1: none)
    std::vector<int32_t> conv_chunks;   // 4 per chunk, placed so that the launch's
                                        // workgroups take them largest first
    std::vector<int32_t> conv_slots;    // 1 + kConvTiles per slot: uid, K[]

    double y_pattern_max = 0.0;   // max 1 - cos(gamma) over all pattern pairs

    int64_t nblocks() const { return (int64_t)blk_col.size(); }
    int64_t nunique() const { return (int64_t)key_delta.size(); }
};

// B-hat between two grids (rows on the auxiliary grid g2, columns on g1) and
// the contraction terms of B-hat^T N_2^-1 B-hat over the stored blocks of g1.
// Tile I of g2 neighbours tile J of g1 when the tile of g1 holding I's centre
// is J or a neighbour of J; blocks are keyed by (band of I in g2, band of J in
// g1, (t_J T_I - t_I T_J) mod T_I T_J).  With g2 = g1 every table equals the
// one-grid table it corresponds to.
struct CrossGeometry {
    int32_t lmax_eff = 0;                 // min(lmax_1, lmax_2)
    std::vector<int32_t> container;       // per tile of g2: tile of g1 holding its centre
    std::vector<int64_t> adj_ptr;         // CSR over tiles I of g2: tiles J of g1, ascending
    std::vector<int32_t> adj_col;
    std::vector<int32_t> adj_uid;         // unique-block id of each (I, J) entry
    std::vector<int32_t> key_band_i, key_band_j;
    std::vector<int64_t> key_delta;
    std::vector<int32_t> rep_i, rep_j;    // a representative (I in g2, J in g1) per key
    std::vector<int64_t> nbr_ptr;         // CSR over tiles J of g1: tiles I of g2, ascending
    std::vector<int32_t> nbr_col;
    std::vector<int64_t> term_ptr;        // per stored block of g1, its terms
    std::vector<Term> terms;              // tile = I of g2 (N_2^-1 pixels [I k^2, (I+1) k^2))
    ClassTables cls;
    std::vector<int32_t> exp_blk, exp_items;   // B-hat blocks (adjacency entries) grouped by unique block
    double y_pattern_max = 0.0;
    int64_t nunique() const { return (int64_t)key_delta.size(); }
};

// A class-grid launch of fewer member tiles than this (32 per CU of the 256)
// takes them from a table in one global largest-first order (geometry.cpp).
constexpr int64_t kShortLaunchTiles = 32 * 256;

// Status codes follow sympix_status. On failure err holds a message.
int build_geometry(int32_t lmax, int32_t k, double margin, Geometry &g, std::string &err);

// The two-hop pattern: every (J, K >= J) whose neighbourhoods intersect, i.e.
// every block of B-hat^T N^-1 B-hat that is not zero when B-hat is local.
int build_two_hop(const Geometry &g, Pattern &p, std::string &err);

// The two-grid tables of B-hat = Y_2 B Y_1^T (g2 auxiliary, g1 the unknowns).
int build_cross(const Geometry &g2, const Geometry &g1, CrossGeometry &x, std::string &err);

}  // namespace sympix
