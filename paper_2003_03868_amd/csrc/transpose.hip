// Block-sparse transpose B = A^T (section "DBCSR library": transpose is one
// of the operations the library provides besides multiply, sum and trace).
// Block (i, j) of A, an m x n row-major block, becomes block (j, i) of B,
// its n x m transpose; B's block rows have A's column sizes and vice versa.
//
// Pattern: blocks are counted per column of A, the counts scanned into B's
// row pointers, and every block placed into its row of B through an atomic
// cursor; each row of B is then sorted by its column (A's row), which makes
// the result independent of the order the atomics ran in.  Values: one
// 64-lane group per block of B copies the transposed block.
#include <algorithm>

#include "bsm_internal.h"

namespace bsm {

namespace {

__global__ void k_t_count(const int64_t *row_ptr, const int32_t *col_idx, int32_t nbrows,
                          unsigned long long *cnt, int32_t *rows) {
    const int32_t i = blockIdx.x;
    if (i >= nbrows) return;
    for (int64_t t = row_ptr[i] + threadIdx.x; t < row_ptr[i + 1]; t += blockDim.x) {
        rows[t] = i;
        atomicAdd(&cnt[col_idx[t]], 1ull);
    }
}

__global__ void k_t_place(const int32_t *col_idx, const int32_t *rows, int64_t nnzb,
                          const int64_t *rp_out, unsigned long long *cursor, int32_t *key,
                          int64_t *src) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nnzb) return;
    const int32_t j = col_idx[t];
    const int64_t p = rp_out[j] + static_cast<int64_t>(atomicAdd(&cursor[j], 1ull));
    key[p] = rows[t];
    src[p] = t;
}

// Insertion sort of each row of B by column (A's row, unique within the row).
__global__ void k_t_sort(const int64_t *rp_out, int32_t nbrows_out, int32_t *key, int64_t *src) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nbrows_out) return;
    const int64_t b = rp_out[j], e = rp_out[j + 1];
    for (int64_t u = b + 1; u < e; ++u) {
        const int32_t k = key[u];
        const int64_t v = src[u];
        int64_t w = u - 1;
        while (w >= b && key[w] > k) {
            key[w + 1] = key[w];
            src[w + 1] = src[w];
            --w;
        }
        key[w + 1] = k;
        src[w + 1] = v;
    }
}

__global__ void k_t_values(const int64_t *src, const int32_t *key, const int32_t *a_col_idx,
                           const int64_t *a_blk_off, const double *a_vals, const int32_t *a_rbs,
                           const int32_t *a_cbs, const int64_t *b_blk_off, double *b_vals,
                           int64_t nnzb) {
    const int64_t p = blockIdx.x;
    if (p >= nnzb) return;
    const int64_t t = src[p];
    const int m = a_rbs[key[p]], n = a_cbs[a_col_idx[t]];
    const double *in = a_vals + a_blk_off[t];
    double *out = b_vals + b_blk_off[p];
    for (int u = threadIdx.x; u < m * n; u += blockDim.x) {
        const int r = u / n, c = u % n;        // in[r][c] -> out[c][r]
        out[c * m + r] = in[u];
    }
}

}  // namespace

int transpose_mat(const Mat &a, Mat **out, hipStream_t s) {
    *out = nullptr;
    if (a.nnzb > INT32_MAX) { set_error("transpose: more than 2^31 blocks"); return BSM_EINVAL; }
    Mat *m = nullptr;
    BSM_TRY(new_mat_sizes(a, true, a, true, &m, s));
    unsigned long long *cnt = nullptr, *cursor = nullptr;
    int32_t *rows = nullptr;
    int st = dalloc(&m->row_ptr, static_cast<size_t>(m->nbrows) + 1, s);
    if (st == BSM_OK) st = dalloc(&m->col_idx, std::max<int64_t>(a.nnzb, 1), s);
    if (st == BSM_OK) st = dalloc(&cnt, static_cast<size_t>(m->nbrows) + 1, s);
    if (st == BSM_OK) st = dalloc(&cursor, static_cast<size_t>(m->nbrows) + 1, s);
    if (st == BSM_OK) st = dalloc(&rows, std::max<int64_t>(a.nnzb, 1), s);
    int64_t *src = nullptr;
    if (st == BSM_OK) st = dalloc(&src, std::max<int64_t>(a.nnzb, 1), s);
    if (st == BSM_OK) {
        hipError_t e = hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (m->nbrows + 1), s);
        if (e == hipSuccess)
            e = hipMemsetAsync(cursor, 0, sizeof(unsigned long long) * (m->nbrows + 1), s);
        if (e != hipSuccess) { set_error("transpose: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st == BSM_OK && a.nbrows > 0 && a.nnzb > 0)
        k_t_count<<<a.nbrows, 64, 0, s>>>(a.row_ptr, a.col_idx, a.nbrows, cnt, rows);
    // counts are non-negative int64 values: scan them as such
    if (st == BSM_OK) st = scan_i64(reinterpret_cast<const int64_t *>(cnt), m->row_ptr, m->nbrows, s);
    if (st == BSM_OK && a.nnzb > 0) {
        k_t_place<<<grid_for(a.nnzb, 256), 256, 0, s>>>(a.col_idx, rows, a.nnzb, m->row_ptr, cursor,
                                                        m->col_idx, src);
        if (m->nbrows > 0)
            k_t_sort<<<grid_for(m->nbrows, 64), 64, 0, s>>>(m->row_ptr, m->nbrows, m->col_idx, src);
    }
    if (st == BSM_OK) {
        m->nnzb = a.nnzb;
        st = compute_blk_off(*m, s);
    }
    if (st == BSM_OK) {
        m->nvalues = a.nvalues;
        st = dalloc(&m->values, std::max<int64_t>(a.nvalues, 1), s);
    }
    if (st == BSM_OK && a.nnzb > 0) {
        k_t_values<<<static_cast<unsigned>(a.nnzb), 64, 0, s>>>(src, m->col_idx, a.col_idx, a.blk_off,
                                                               a.values, a.rbs, a.cbs, m->blk_off,
                                                               m->values, a.nnzb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_error("transpose: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    dfree(cnt, s);
    dfree(cursor, s);
    dfree(rows, s);
    dfree(src, s);
    if (st != BSM_OK) { free_mat(m, s); return st; }
    *out = m;
    return BSM_OK;
}

}  // namespace bsm
