// Retained symbolic state of one multiply and its numeric-only repetition.
//
// A multiply's symbolic phase (C pattern, product stacks, sorted work lists,
// the filter's keep-set and the compaction maps) depends only on the block
// patterns of A, B and C_in.  When an iteration reuses the same patterns with
// new values, replay_multiply runs just the numeric kernels: optional operand
// packing, the block products, a check that the filter keeps exactly the same
// blocks, and a values-only gather into the filtered layout.  It launches
// kernels only (no allocation, copy or wait), so it can be captured into a
// hipGraph.
#pragma once

#include <vector>

#include "smm.h"

namespace bsm {

constexpr int kFlagPattern = 2;   // the filter would keep a different block set

enum MulOpKind { kOpVariant = 0, kOpClass = 1, kOpRt = 2, kOpLowp = 3, kOpQuad = 4, kOpMQuad = 5 };

// One block-product launch of a multiply.
struct MulOp {
    int kind = kOpVariant;
    int id = 0;          // kernel variant (kOpVariant) or (m, n) class (kOpClass)
    SmmParams prm{};     // kOpRt
    SmmArgs a{};         // plan-owned symbolic arrays; value pointers patched per run
};

int run_op(const MulOp &op, hipStream_t s);

struct MulPlan {
    hipStream_t s = nullptr;          // stream its memory is released on
    double alpha = 0.0, beta = 0.0, eps = 0.0;
    int norm = 0, prec = 0;
    bool use_c = false, same_ab = false;
    // operand sizes the plan was made for
    int64_t a_nnzb = 0, b_nnzb = 0, cin_nnzb = 0, a_nval = 0, b_nval = 0;
    // the product before (u) and after the filter
    int64_t nnzb_u = 0, nval_u = 0, nnzb = 0, nval = 0;
    bool compacted = false;           // the filter dropped blocks
    double flops = 0.0;
    int64_t nprod = 0;
    int64_t *c_row_ptr_u = nullptr;   // unfiltered pattern (plan-owned)
    int32_t *c_col_u = nullptr;
    int64_t *c_blk_off_u = nullptr;
    double *c_vals_u = nullptr;       // unfiltered values when compacted
    double *sq = nullptr, *mx = nullptr;  // block norms of the product
    int64_t *kidx = nullptr, *koff = nullptr;   // keep scan and kept offsets
    uint32_t *apk = nullptr, *bpk = nullptr;    // packed reduced-precision operands
    std::vector<void *> owned;
    std::vector<MulOp> ops;
};

// A, B and Cin (NULL when beta == 0) must have the patterns the plan was made
// for; their values may differ.  Writes the filtered product (p.nval values in
// the plan's filtered layout) to out, which must not alias A, B or Cin.  flags
// collects kFlagNonFinite and kFlagPattern; the caller clears it beforehand.
int replay_multiply(MulPlan &p, const Mat &A, const Mat &B, const Mat *Cin, double *out,
                    int *flags, hipStream_t s);

// Rebuild m from a replay's unfiltered product (vals_u: the plan's
// unfiltered layout; may be m.values) and filter it anew.  Used when the
// filter of a replay keeps other blocks than the plan recorded: the product
// itself is still exact, only its compaction changes.
int refilter(const MulPlan &p, const double *vals_u, Mat &m, hipStream_t s);

// *f = 0 by a kernel (usable inside a captured graph).
int zero_flag(int *f, hipStream_t s);

// Device comparison of two block patterns with the same nbrows and nnzb:
// sets *diff (device int, cleared here) to 1 when they differ.
int pattern_differs(const int64_t *rp_a, const int32_t *ci_a, const int64_t *rp_b,
                    const int32_t *ci_b, int32_t nbrows, int64_t nnzb, int *diff, hipStream_t s);

}  // namespace bsm
