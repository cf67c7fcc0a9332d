// Matrix sum C = alpha A + beta B + gamma I with the norm filter (the sum
// among the DBCSR matrix operations), used by the higher-order sign
// iterations.  Pattern = pattern(A) union pattern(B), plus the diagonal
// blocks when gamma != 0; per element v = alpha a + beta b (absent blocks
// read as zero), then + gamma on the diagonal.
#include <cmath>

#include "bsm_internal.h"

namespace bsm {

// One thread per block row: merge A's and B's column lists (and the
// diagonal).  Count pass (cnt != NULL) or fill pass (col, src_a, src_b).
__global__ void k_add_rows(const int64_t *a_rp, const int32_t *a_ci, const int64_t *b_rp,
                           const int32_t *b_ci, int32_t nbrows, int32_t nbcols, int diag,
                           int64_t *cnt, const int64_t *row_ptr, int32_t *col, int64_t *src_a,
                           int64_t *src_b) {
    const int64_t i64 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i64 >= nbrows) return;
    const int32_t i = static_cast<int32_t>(i64);
    int64_t ta = a_rp[i], tb = b_rp ? b_rp[i] : 0;
    const int64_t ea = a_rp[i + 1], eb = b_rp ? b_rp[i + 1] : 0;
    bool done_diag = !diag;
    int64_t n = 0, w = row_ptr ? row_ptr[i] : 0;
    for (;;) {
        const int32_t ja = ta < ea ? a_ci[ta] : nbcols;
        const int32_t jb = tb < eb ? b_ci[tb] : nbcols;
        const int32_t jd = done_diag ? nbcols : i;
        int32_t j = ja < jb ? ja : jb;
        if (jd < j) j = jd;
        if (j >= nbcols) break;
        if (j == i) done_diag = true;
        const int64_t sa = (ja == j) ? ta++ : -1;
        const int64_t sb = (jb == j) ? tb++ : -1;
        if (row_ptr) {
            col[w + n] = j;
            src_a[w + n] = sa;
            src_b[w + n] = sb;
        }
        ++n;
    }
    if (cnt) cnt[i] = n;
}

// One wave per output block: values and the block's filter norms.
__global__ void __launch_bounds__(64)
k_add_vals(const int32_t *col, const int64_t *row_ptr, int32_t nbrows, const int64_t *src_a,
           const int64_t *src_b, const int64_t *out_off, const int64_t *a_off, const double *a_vals,
           const int64_t *b_off, const double *b_vals, const int32_t *rbs, const int32_t *cbs,
           double alpha, double beta, double gamma, double *out, double *sq, double *mx,
           int64_t nnzb) {
    const int64_t d = blockIdx.x;
    if (d >= nnzb) return;
    // owning row: binary search in row_ptr
    int32_t lo = 0, hi = nbrows - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= d) lo = mid; else hi = mid - 1;
    }
    const int32_t i = lo, j = col[d];
    const int m = rbs[i], n = cbs[j];
    const int64_t sa = src_a[d], sb = src_b ? src_b[d] : -1;
    double s2 = 0.0, mxv = 0.0;
    for (int e = threadIdx.x; e < m * n; e += 64) {
        double v = sa >= 0 ? alpha * a_vals[a_off[sa] + e] : 0.0;
        if (sb >= 0) v = v + beta * b_vals[b_off[sb] + e];
        if (i == j && (e / n) == (e % n)) v = v + gamma;
        out[out_off[d] + e] = v;
        s2 += v * v;
        mxv = fmax(mxv, fabs(v));
    }
    for (int o = 32; o > 0; o >>= 1) {
        s2 += __shfl_xor(s2, o, 64);
        mxv = fmax(mxv, __shfl_xor(mxv, o, 64));
    }
    if (threadIdx.x == 0) {
        sq[d] = s2;
        mx[d] = mxv;
    }
}

int add_mat(double alpha, const Mat &a, double beta, const Mat *b, double gamma, double eps,
            int norm, Mat **out, hipStream_t s) {
    *out = nullptr;
    if (b && (b->nbrows != a.nbrows || b->nbcols != a.nbcols || b->h_rbs != a.h_rbs ||
              b->h_cbs != a.h_cbs)) {
        set_error("add: A and B must have the same block sizes");
        return BSM_EINVAL;
    }
    if (gamma != 0.0 && (a.nbrows != a.nbcols || a.h_rbs != a.h_cbs)) {
        set_error("add: gamma != 0 needs a square block matrix with square diagonal blocks");
        return BSM_EINVAL;
    }
    if (!(eps >= 0.0) || !std::isfinite(eps)) { set_error("add: eps_filter must be finite and >= 0"); return BSM_EINVAL; }
    if (norm != BSM_NORM_FROB && norm != BSM_NORM_MAXABS) { set_error("add: unknown norm"); return BSM_EINVAL; }
    if (!std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(gamma)) {
        set_error("add: alpha, beta and gamma must be finite");
        return BSM_EINVAL;
    }
    Mat *m = nullptr;
    BSM_TRY(alloc_like_sizes(a, a, &m, s));
    const int32_t nbr = a.nbrows;
    const int diag = gamma != 0.0 ? 1 : 0;
    int64_t *src_a = nullptr, *src_b = nullptr;
    double *sq = nullptr, *mx = nullptr;
    int st = dalloc(&m->row_ptr, nbr + 1, s);
    int64_t nnzb = 0, nv = 0;
    auto read1 = [&](const int64_t *d, int64_t *h) -> int {
        hipError_t e = hipMemcpyAsync(h, d, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { set_error("add: %s", hipGetErrorString(e)); return BSM_EDEVICE; }
        return BSM_OK;
    };
    const int64_t *b_rp = b ? b->row_ptr : nullptr;
    const int32_t *b_ci = b ? b->col_idx : nullptr;
    if (st == BSM_OK && nbr > 0) {
        k_add_rows<<<grid_for(nbr, 128), 128, 0, s>>>(a.row_ptr, a.col_idx, b_rp, b_ci, nbr, a.nbcols,
                                                      diag, m->row_ptr, nullptr, nullptr, nullptr,
                                                      nullptr);
        st = scan_i64(m->row_ptr, m->row_ptr, nbr, s);
        if (st == BSM_OK) st = read1(m->row_ptr + nbr, &nnzb);
    } else if (st == BSM_OK) {
        hipError_t e = hipMemsetAsync(m->row_ptr, 0, sizeof(int64_t), s);
        if (e != hipSuccess) { set_error("add: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st == BSM_OK) st = dalloc(&m->col_idx, nnzb, s);
    if (st == BSM_OK) st = dalloc(&src_a, nnzb, s);
    if (st == BSM_OK) st = dalloc(&src_b, nnzb, s);
    if (st == BSM_OK && nbr > 0)
        k_add_rows<<<grid_for(nbr, 128), 128, 0, s>>>(a.row_ptr, a.col_idx, b_rp, b_ci, nbr, a.nbcols,
                                                      diag, nullptr, m->row_ptr, m->col_idx, src_a,
                                                      src_b);
    m->nnzb = nnzb;
    if (st == BSM_OK) st = compute_blk_off(*m, s);
    if (st == BSM_OK) st = read1(m->blk_off + nnzb, &nv);
    m->nvalues = nv;
    if (st == BSM_OK) st = dalloc(&m->values, nv, s);
    if (st == BSM_OK) st = dalloc(&sq, nnzb, s);
    if (st == BSM_OK) st = dalloc(&mx, nnzb, s);
    if (st == BSM_OK && nnzb > 0) {
        k_add_vals<<<static_cast<unsigned>(nnzb), 64, 0, s>>>(
            m->col_idx, m->row_ptr, nbr, src_a, b ? src_b : nullptr, m->blk_off, a.blk_off, a.values,
            b ? b->blk_off : nullptr, b ? b->values : nullptr, a.rbs, a.cbs, alpha, beta, gamma,
            m->values, sq, mx, nnzb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_error("add kernel: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    int64_t after = nnzb;
    if (st == BSM_OK && eps > 0.0) st = compact_by_norm(*m, sq, mx, eps, norm, s, &after);
    dfree(src_a, s); dfree(src_b, s); dfree(sq, s); dfree(mx, s);
    if (st != BSM_OK) { free_mat(m, s); return st; }
    *out = m;
    return BSM_OK;
}

}  // namespace bsm
