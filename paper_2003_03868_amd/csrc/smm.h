// Numeric phase (product-stack execution); see smm.hip.
#pragma once

#include "bsm_internal.h"

namespace bsm {

constexpr int kFlagNonFinite = 1;

// Parameters of the tunable run-time-shape kernel (smm_rt.hip).
struct SmmParams {
    int32_t family;    // 0: 16x16x4 FP64 MFMA, 1: 4x4x4 FP64 MFMA, 2: per-class kernel,
                       // 3: compile-time-shape kernel (m = n = k in {5,13,23,26,32})
    int32_t wpg;       // C blocks (wavefronts) per workgroup: 1, 2, 4
    int32_t prefetch;  // 1: prefetch the next product's operands
    int32_t reserved;
};

// Block-product kernel variants.
enum SmmVariant {
    kSmmF64M16 = 0,   // V_MFMA_F64_16X16X4_F64, 16 x 16 tiles
    kSmmF64M4 = 1,    // V_MFMA_F64_4X4X4_4B_F64, 4 x 4 tiles, run-time shapes
    kSmmF64Fixed = 2, // same instruction, compile-time uniform shapes (default
                      // for uniform sizes)
    kSmmF64Fused = 3, // persistent kernel: all (m, n) classes of a chunk in one
                      // launch, cost-sorted work queue, run-time shapes
    kSmmF64Class = 4, // one launch per (m, n) class of {5,13,23,26}^2 with an
                      // (m, n)-specialised kernel, run-time k
    kSmmF64Tuned = 5, // tunable run-time-shape kernel, parameters from the table
    kSmmF64Quad = 6,  // compile-time uniform shapes, one workgroup per 2 x 2 quad of
                      // C blocks (default for uniform sizes 5, 6, 13, 23, 26, 32)
    kSmmF64MQuad = 7, // mixed sizes in {5, 13, 23, 26}: 2 x 2 groups over paired rows and
                      // columns of equal size, every class in one persistent launch
};

struct SmmArgs {
    int64_t c0;                 // first C block of this launch
    int64_t nC;                 // C blocks in this launch
    const int64_t *worklist;    // C block of work item c0 + item (NULL: identity)
    const int64_t *seg;         // [nC+1] product segments, launch-relative
    const int32_t *stk_a;       // A block index per product
    const int32_t *stk_b;       // B block index per product
    const int32_t *c_row;       // block row of every C block
    const int32_t *c_col;       // block column of every C block
    const int64_t *c_blk_off;   // value offset of every C block
    double *c_vals;             // C values (written)
    const int32_t *c_rbs, *c_cbs;
    const int32_t *a_col_idx;
    const int64_t *a_blk_off;
    const double *a_vals;
    const int32_t *k_size;      // A column block sizes
    const int64_t *b_blk_off;
    const double *b_vals;
    const uint32_t *a_pk, *b_pk;  // packed reduced-precision operands (prec != FP64)
    int64_t a_pk_n, b_pk_n;       // elements packed in a_pk, b_pk (three-term split: the
                                  // lo parts follow the first a_pk_n words as uint16)
    const int64_t *cin_map;     // C_in block of every C block or -1; NULL when beta == 0
    const int64_t *cin_blk_off;
    const double *cin_vals;
    double alpha, beta;
    double *sq_out;             // sum of squares of every C block
    double *mx_out;             // max |x| of every C block
    int *flags;                 // kFlagNonFinite
    int32_t max_m, max_n, max_k;
    int32_t uni_m, uni_n, uni_k;  // uniform block sizes, 0 if mixed
    int32_t fused_ok;             // every block size is in {5, 13, 23, 26}
    int32_t pad_;
    int32_t prec;               // bsm_precision
    unsigned long long *counter;  // work counter of the persistent kernel (NULL: allocated per launch)
    // group kernel: GR x GC groups of C blocks (2 x 2: quads) with merged product lists
    int64_t n_quads;            // groups
    const int64_t *n_quads_dev; // FP64 group kernels: the group count in device memory (the
                                // launch then covers up to n_quads groups); NULL: n_quads
    const int64_t *q_cblk;      // [GR GC n_quads] C block (r, c) of the group at GC r + c, or -1
    const int64_t *q_seg;       // [n_quads + 1] entry segments
    const int4 *q_ent;          // ceil((GR + GC) / 4) int4 per entry: A(row 0..GR-1) then
                                // B(col 0..GC-1) block indices, -1 where absent
    const int64_t *q_order;     // group of work item i (NULL: identity)
    int32_t q_gr, q_gc;         // group shape
    const int32_t *q_pm;        // product mask per entry (bit GC r + c), NULL: all products
};

int smm_launch(const SmmArgs &a, int variant, hipStream_t s);
// Requested block-product variant (kSmmF64Quad unless BSM_SMM_VARIANT says otherwise).
int smm_variant();
bool smm_fixed_available(int m, int n, int k);
int launch_fixed(const SmmArgs &a, int m, unsigned grid, hipStream_t s);
int class_of_size(int b);                       // 0..3 for 5, 13, 23, 26; else -1
int launch_class(const SmmArgs &a, int cls, hipStream_t s);   // cls = 4*class(m)+class(n)

// Tunable run-time-shape kernels (smm_rt.hip) and the tuning table (tune.hip).
int launch_rt(const SmmArgs &a, const SmmParams &prm, hipStream_t s);
bool table_lookup(int m, int n, int k, SmmParams *out);    // k = 0: mixed k
void table_set(int count, const int32_t *mnk, const SmmParams *prm);   // count < 0 clears
int smm_bench(int m, int n, int k, int64_t n_c, int per_c, int n_prm, const SmmParams *prm,
              int reps, double *ms_out, hipStream_t s);

// Quad kernel (smm_quad.hip): uniform m = n = k in {5, 6, 13, 23, 26, 32}.
bool smm_quad_available(int m, int n, int k);
// Group shape for uniform block size m: 2 x 2 (quads) unless BSM_QUAD_GROUP
// asks for 4 (4 x 4) or 42 (4 x 2, size 23) and m has that kernel.
void quad_shape(int m, int *gr, int *gc);
int launch_quad(const SmmArgs &a, hipStream_t s);
// Mixed-size groups (smm_mquad.hip): one persistent launch over a.n_quads
// groups built with paired rows and columns (a.counter: work counter).
int launch_mquad(const SmmArgs &a, hipStream_t s);
// Work order of the mixed-size groups (largest m n first, group order within
// a class) into order[a.n_quads]; rank_scratch holds a.n_quads bytes (with
// a.n_quads_dev, the first *a.n_quads_dev groups are ordered).
int mquad_order(const SmmArgs &a, int8_t *rank_scratch, int64_t *order, hipStream_t s);

// Reduced-precision products (smm_lowp.hip).
int pack_lowp(const double *v, int64_t n, uint32_t *out, int prec, hipStream_t s);
// 32-bit words of the packed form of n elements (lowp_words(n, prec) >= n).
inline int64_t lowp_words(int64_t n, int prec) {
    return prec == BSM_SPLIT_BF16X3 ? n + (n + 1) / 2 : n;
}
bool smm_lowp_available(int m, int n, int k);
int smm_launch_lowp(const SmmArgs &a, hipStream_t s);
int launch_lowp_quad(const SmmArgs &a, hipStream_t s);   // quads, uniform sizes as above

}  // namespace bsm
