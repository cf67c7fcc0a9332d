// Symbolic phase (pattern of C and product stacks); see symbolic.hip.
#pragma once

#include "bsm_internal.h"

namespace bsm {

// Rows of a C block row whose block count exceeds this are stacked in
// windows of this many C blocks (LDS counters per window).
constexpr int kStackWindow = 4096;
// Largest block-column count the LDS bitmaps support.
constexpr int32_t kMaxBlockCols = 131072;

struct SymArgs {
    int32_t nbrows, nbcols;              // block grid of C
    const int64_t *a_row_ptr;
    const int32_t *a_col_idx;
    const int64_t *b_row_ptr;
    const int32_t *b_col_idx;
    const int32_t *k_size;               // A column block sizes (= B row sizes)
    const int32_t *c_rbs, *c_cbs;        // C block sizes
    int use_c;                           // include C_in's pattern (beta != 0)
    const int64_t *c_in_row_ptr;
    const int32_t *c_in_col_idx;
};

// Tiled order of the C blocks (bands of `rb` block rows, column bands of
// tile_cols() columns); writes worklist[c] for every C block.
// wb < 1: tile_cols() block columns per column band.
int tile_order(const int64_t *c_row_ptr, const int32_t *c_col_idx, int32_t nbrows,
               int32_t nbcols, int rb, int64_t *worklist, hipStream_t s, int wb = 0);
// Tile shape (BSM_TILE_ROWS / BSM_TILE_COLS override the defaults 16 / 32;
// BSM_TILE_ROWS=1 with BSM_TILE_COLS >= nbcols gives plain CSR order).
int tile_rows();
int tile_cols();

// Bucket sort of the work list entries [c0, c0+n) (see symbolic.hip);
// hist_host (64 entries, may be NULL) receives the bucket sizes (waits).
constexpr int kKeyCost = 0, kKeyClass = 1;
int sort_worklist(const int64_t *wl_in, int64_t *wl_out, int64_t c0, int64_t n, int mode,
                  const int32_t *c_row, const int32_t *c_col, const int32_t *rbs,
                  const int32_t *cbs, const int64_t *seg, int64_t *hist_host, hipStream_t s);

// GR x GC groups of C blocks (2 x 2: quads) and their merged entry lists,
// straight from the patterns of A, B and the unfiltered C (quad.hip), over
// the row groups of block rows [r0, r1) (r0 a multiple of GR).  quad_pairs:
// cnt[R] = groups of row group R.  quad_stack count pass (fill = false),
// with q_off = scanned group counts: q_cblk[GR GC q + GC r + c] = C block
// (GR R + r, GC Q + c) or -1, q_col[q] = Q and e_off[q nseg + s] = entries
// of group q with k in segment s; fill pass (e_off scanned): entry n of
// segment s of group q at ent[NE (e_off[q nseg + s] + n)] with
// NE = ceil((GR + GC) / 4), ascending k, so each group's entries are
// contiguous and in ascending k.  Segment s covers k in [s kseg, (s + 1) kseg);
// one workgroup per (row group, segment).  Shapes: 2x2, 4x4, 4x2.
struct QuadSymArgs {
    int32_t r0, r1, nbcols;
    int32_t gr, gc;              // group shape: rows x columns (2 x 2: quads)
    int32_t nseg, kseg;          // the k range split into nseg segments of kseg values
    const int64_t *a_row_ptr;
    const int32_t *a_col_idx;
    const int64_t *b_row_ptr;
    const int32_t *b_col_idx;
    const int64_t *c_row_ptr;    // unfiltered C pattern
    const int32_t *c_col_idx;
    const int64_t *q_off;
    int64_t *q_cblk;
    int32_t *q_col;              // column group Q of every group (count pass)
    int64_t *e_off;              // [n_groups nseg + 1]: count pass, entries per (group, segment);
                                 // fill pass, their scanned offsets (group-major)
    int4 *ent;                   // ceil((gr + gc) / 4) int4 per entry
    // product-level norm screening (tau2 > 0): products with
    // a_sq[A block] * b_sq[B block] < tau2 are left out of the entries; the
    // fill pass writes each entry's product mask (bit GC r + c) to pm and
    // adds the kept products to *kept
    const double *a_sq, *b_sq;
    double tau2;
    int32_t *pm;
    unsigned long long *kept;
    // mixed block sizes (map = 1; 2 x 2 only): groups over paired rows and
    // columns of equal size instead of consecutive ones
    int32_t map;
    int32_t g0;                  // first row group of this chunk
    int64_t ngroups;             // row groups of this chunk
    int32_t ncg;                 // column groups
    const int32_t *rg;           // [2 G] rows of row group g (second -1 for a single row)
    const int32_t *cgrp;         // [nbcols] column group of column j
    const int32_t *cslot;        // [nbcols] slot (0 or 1) of column j in its group
    const int32_t *cmap;         // [2 ncg] columns of column group Q (second -1 for one)
};
// Pairs of equal-size block rows (within bands of kPairBand rows) and of
// equal-size block columns for the mixed-size groups (quad.hip): rg[2g],
// rg[2g + 1] are the rows of row group g (second -1 for a single row),
// band_g0[b] the first row group of band b (band_g0.back(): all row groups),
// cmap[2Q], cmap[2Q + 1] the columns of column group Q, cgrp[j] and cslot[j]
// column j's group and slot.
constexpr int32_t kPairBand = 32;
struct MixedPairs {
    std::vector<int32_t> rg, band_g0, cgrp, cslot, cmap;
};
void mixed_pairs(const std::vector<int32_t> &rbs, const std::vector<int32_t> &cbs, MixedPairs *mp);

// k segments of the group lists' walk for nbk block columns of A.
int32_t quad_ksegments(int32_t nbk);
int quad_pairs(const QuadSymArgs &q, int64_t *cnt, hipStream_t s);
int quad_stack(const QuadSymArgs &q, bool fill, hipStream_t s);
// starts[g] = seg_off[g nseg] for g in [0, n_groups]: entry offsets per group.
int quad_seg_starts(const int64_t *seg_off, int32_t nseg, int64_t n_groups, int64_t *starts,
                    hipStream_t s);

int sym_count(const SymArgs &a, int64_t *c_cnt, int64_t *c_nval, int64_t *p_cnt, double *flops,
              hipStream_t s);
int sym_pattern(const SymArgs &a, const int64_t *c_row_ptr, int32_t *c_col_idx, int32_t *c_row,
                int64_t *cin_map, hipStream_t s);
int sym_stack(const SymArgs &a, int32_t r0, int32_t r1, const int64_t *c_row_ptr,
              const int64_t *p_row_ptr, int64_t *seg, int32_t *stk_a, int32_t *stk_b,
              hipStream_t s);

}  // namespace bsm
