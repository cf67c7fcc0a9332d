// Internal declarations shared by the bsm HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bsm.h"

namespace bsm {

constexpr int kMaxBlock = 32;          // largest supported block edge
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kXcds = 8;               // MI355X: 8 accelerator complex dies

// Device-resident blocked-CSR matrix.  All pointers are device memory.
struct Mat {
    int device = 0;
    int32_t nbrows = 0, nbcols = 0;
    int64_t nnzb = 0, nvalues = 0, nrows = 0, ncols = 0;
    std::vector<int32_t> h_rbs, h_cbs;       // host copies of the block sizes
    int32_t max_rbs = 0, max_cbs = 0;
    int32_t uni_r = 0, uni_c = 0;            // uniform block size, 0 if mixed
    int32_t *rbs = nullptr, *cbs = nullptr;  // [nbrows], [nbcols]
    int64_t *roff = nullptr, *coff = nullptr;// scalar offsets [nb+1]
    int64_t *row_ptr = nullptr;              // [nbrows+1]
    int32_t *col_idx = nullptr;              // [nnzb]
    int64_t *blk_off = nullptr;              // [nnzb+1] value offsets
    double *values = nullptr;                // [nvalues]
    hipStream_t stream = nullptr;            // last stream the handle was used on
};

// ------------------------------------------------------------ error state
void set_error(const char *fmt, ...);
void clear_error();

// The block-product kernel most recently launched by this thread, as written
// at its launch (BSM_LAUNCH records it; bsm_last_smm_kernel reports it).
void note_kernel(const char *launch_text);
void note_kernelf(const char *fmt, ...);   // the same, formatted (template arguments of a template)
const char *last_kernel();
#define BSM_ID(...) __VA_ARGS__
// BSM_LAUNCH((kernel<args>), grid, block, lds, stream)(kernel arguments)
#define BSM_LAUNCH(KER, G, ...) BSM_ID KER<<<(::bsm::note_kernel(#KER), (G)), __VA_ARGS__>>>

#define BSM_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            ::bsm::set_error("%s failed: %s (%s:%d)", #expr,                   \
                             hipGetErrorString(e_), __FILE__, __LINE__);       \
            return BSM_EDEVICE;                                                \
        }                                                                      \
    } while (0)

#define BSM_TRY(expr)                                                          \
    do {                                                                       \
        int s_ = (expr);                                                       \
        if (s_ != BSM_OK) return s_;                                           \
    } while (0)

// --------------------------------------------------------------- memory
// Device allocations from the library's caching allocator (util.hip): blocks
// freed on a stream are reused by later allocations on the same stream.
int dalloc_bytes(void **p, size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s);
template <class T>
inline int dalloc(T **p, size_t n, hipStream_t s) {
    return dalloc_bytes(reinterpret_cast<void **>(p), n * sizeof(T), s);
}

void free_mat_arrays(Mat &m, hipStream_t s);   // values/pattern (not sizes)
void free_mat(Mat *m, hipStream_t s);

// ------------------------------------------------------------- helpers
inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (1ll << 30)) g = 1ll << 30;
    return static_cast<unsigned>(g);
}

// Exclusive scan of n int64 values into out[0..n]; out[n] = total.
// `in` and `out` may alias.  Work space is allocated on the stream.
int scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
// The same with caller-provided work space of scan_ws_words(n) words (no
// allocation, no copy: capturable into a graph).
int64_t scan_ws_words(int64_t n);
int scan_i64_ws(const int64_t *in, int64_t *out, int64_t n, int64_t *ws, hipStream_t s);

// Block value offsets blk_off[nnzb+1] from row_ptr/col_idx/block sizes.
int compute_blk_off(Mat &m, hipStream_t s);

// Device check of canonical form; returns BSM_EINVAL with a message.
int validate_pattern(const Mat &m, hipStream_t s);

// ---------------------------------------------------------- multiply core
// Symbolic state of one multiply kept for numeric-only repetitions with the
// same operand patterns (graph replay in the sign iteration); plan.hip.
struct MulPlan;
void free_plan(MulPlan *p);

// Sizes of one multiply's symbolic results (to size fixed-capacity buffers).
struct MulSizes {
    int64_t nnzb_u = 0;      // C blocks before the filter
    int64_t nnzb = 0;        // C blocks after the filter
    int64_t nval_u = 0;      // C scalars before the filter
    int64_t nval = 0;        // C scalars after the filter
    int64_t n_groups = 0;    // groups of C blocks of the group kernel, over all chunks
    int64_t n_entries = 0;   // their entries
    bool groups = false;     // an FP64 group kernel did the products (uniform sizes, or
                             // mixed sizes in one launch)
};

// plan (may be NULL): on success receives the retained symbolic state.
// tau > 0: product-level norm screening (terms with ||A_ik||^2 ||B_kj||^2 <
// tau^2 left out; FP64 group kernel only).  sizes (may be NULL): receives
// the sizes above.
int multiply(double alpha, Mat &A, Mat &B, double beta, Mat &C, double eps,
             int norm, int prec, bsm_mult_stats *stats, hipStream_t s,
             MulPlan **plan = nullptr, double tau = 0.0, MulSizes *sizes = nullptr);
int filter_inplace(Mat &m, double eps, int norm, hipStream_t s);

// Reductions (reduce.hip)
int block_sqnorms(const Mat &m, double *out, hipStream_t s);
int trace(const Mat &m, double *out, hipStream_t s);
int sqdist_identity(const Mat &m, double shift, double *out, hipStream_t s);
// The same sum into a device double, partial sums in fixed device memory
// (no allocation, no wait); BSM_ECAPACITY beyond 2^20 block rows.
int sqdist_identity_noalloc(const Mat &m, double shift, double *out_dev, hipStream_t s);
int inf_norm(const Mat &m, double mu, double *out, hipStream_t s);
int shift_scale(const Mat &a, double mu, double scale, Mat **out, hipStream_t s);
int copy_mat(const Mat &a, Mat **out, hipStream_t s);
// C = alpha A + beta B + gamma I (b may be NULL), filtered, as a new matrix (add.hip).
int add_mat(double alpha, const Mat &a, double beta, const Mat *b, double gamma, double eps,
            int norm, Mat **out, hipStream_t s);
// A matrix without a pattern whose block rows have the sizes of proto_rows'
// rows and whose block columns those of proto_cols' columns.
int alloc_like_sizes(const Mat &proto_rows, const Mat &proto_cols, Mat **out, hipStream_t s);
// The same with either side taken transposed: rows from r's columns
// (r_cols), columns from c's rows (c_rows).
int new_mat_sizes(const Mat &r, bool r_cols, const Mat &c, bool c_rows, Mat **out, hipStream_t s);
// B = A^T as a new matrix (transpose.hip).
int transpose_mat(const Mat &a, Mat **out, hipStream_t s);

// Compaction after the filter (reduce.hip).  keep (may be NULL): instead of
// freeing them, hand over the keep scan kidx[n+1], the kept-value offsets
// koff[n+1] and the unfiltered arrays of m (col_idx, blk_off, values).
struct CompactKeep {
    int64_t *kidx = nullptr, *koff = nullptr;
    int64_t *row_ptr = nullptr, *blk_off = nullptr;
    int32_t *col_idx = nullptr;
    double *values = nullptr;
    bool compacted = false;      // false: nothing was dropped, m unchanged
};
int compact_by_norm(Mat &m, const double *sq, const double *mx, double eps, int norm,
                    hipStream_t s, int64_t *nnzb_after, CompactKeep *keep = nullptr);

// ||A - shift I||_F^2 into a device scalar (part: nbrows doubles of scratch).
int sqdist_identity_dev(const Mat &m, double shift, double *part, double *d_out, hipStream_t s);

}  // namespace bsm
