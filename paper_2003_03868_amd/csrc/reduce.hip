// Whole-matrix reductions (block norms, trace, ||A - sI||_F^2, infinity
// norm), the norm filter with compaction, and the shifted/scaled copy used
// for X_0 = (H - mu I)/s and P = (I - X)/2.  All reductions are FP64 and sum
// in a fixed order, so repeated calls give identical bits.
#include <mutex>

#include "bsm_internal.h"

namespace bsm {

constexpr int kRedThreads = 256;

// Fixed device memory for the residual reduction that allocates nothing
// (sqdist_identity_noalloc): one partial sum per block row, at most
// kNoAllocMaxRows rows (8 MiB).  Every device the library runs on holds its
// own copy until the process ends; calls on one device share it, so calls
// that overlap on one device race.  Host code never passes the symbol itself
// to a kernel: its device address comes from hipGetSymbolAddress, taken once
// per device with that device current.
constexpr int64_t kNoAllocMaxRows = int64_t{1} << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocMaxRows];

static std::mutex g_scratch_mu;
static double *g_scratch_dev[kNoAllocMaxDevices] = {};

static int scratch_address(double **out) {
    int dev = 0;
    BSM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        set_error("device %d is beyond the %d devices of the fixed scratch table", dev,
                  kNoAllocMaxDevices);
        return BSM_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the fixed scratch failed: %s", hipGetErrorString(e));
            return BSM_EDEVICE;
        }
        g_scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[dev];
    return BSM_OK;
}

__device__ inline double wsum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double wmax(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Deterministic single-workgroup sum (or max) of n partial values.
__global__ void __launch_bounds__(1024) k_reduce_final(const double *part, int64_t n, double *out,
                                                       int take_max) {
    __shared__ double sh[1024];
    double v = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += 1024) v = take_max ? fmax(v, part[t]) : v + part[t];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            sh[threadIdx.x] = take_max ? fmax(sh[threadIdx.x], sh[threadIdx.x + w])
                                       : sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

static int reduce_to_host(const double *part, int64_t n, int take_max, double *host_out,
                          hipStream_t s) {
    double *d_out = nullptr;
    BSM_TRY(dalloc(&d_out, 1, s));
    k_reduce_final<<<1, 1024, 0, s>>>(part, n, d_out, take_max);
    BSM_HIP(hipGetLastError());
    BSM_HIP(hipMemcpyAsync(host_out, d_out, sizeof(double), hipMemcpyDeviceToHost, s));
    BSM_HIP(hipStreamSynchronize(s));
    dfree(d_out, s);
    return BSM_OK;
}

// ------------------------------------------------------------ block norms

// One wavefront per stored block: sum of squares and max |x|.
__global__ void __launch_bounds__(kRedThreads)
k_block_norms(const int64_t *blk_off, const double *vals, int64_t nnzb, double *sq, double *mx) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * (kRedThreads / kWave) +
                      threadIdx.x / kWave;
    if (t >= nnzb) return;
    const int lane = threadIdx.x % kWave;
    double s = 0.0, m = 0.0;
    for (int64_t e = blk_off[t] + lane; e < blk_off[t + 1]; e += kWave) {
        const double x = vals[e];
        s += x * x;
        m = fmax(m, fabs(x));
    }
    s = wsum(s);
    m = wmax(m);
    if (lane == 0) {
        if (sq) sq[t] = s;
        if (mx) mx[t] = m;
    }
}

int block_sqnorms(const Mat &m, double *out, hipStream_t s) {
    if (m.nnzb == 0) return BSM_OK;
    k_block_norms<<<grid_for(m.nnzb, kRedThreads / kWave), kRedThreads, 0, s>>>(
        m.blk_off, m.values, m.nnzb, out, nullptr);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// ------------------------------------------------------ filter/compaction

__global__ void k_keep(const double *sq, const double *mx, const int64_t *blk_off, int64_t n,
                       double eps, int norm, int64_t *keep, int64_t *ksize) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const bool k = (norm == BSM_NORM_MAXABS) ? !(mx[t] < eps) : !(sq[t] < eps * eps);
    keep[t] = k ? 1 : 0;
    ksize[t] = k ? (blk_off[t + 1] - blk_off[t]) : 0;
}

__global__ void k_compact_rows(const int64_t *row_ptr, const int64_t *kidx, int32_t nbrows,
                               int64_t *new_row_ptr) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i <= nbrows) new_row_ptr[i] = kidx[row_ptr[i]];
}

// One workgroup per block: copy a kept block to its new place.
__global__ void __launch_bounds__(64)
k_compact_blocks(const int64_t *kidx, const int64_t *koff, const int32_t *col_idx,
                 const int64_t *blk_off, const double *vals, int64_t n, int32_t *new_col,
                 int64_t *new_off, double *new_vals) {
    const int64_t t = blockIdx.x;
    if (t >= n) return;
    const int64_t d = kidx[t];
    if (kidx[t + 1] == d) return;   // dropped
    const int64_t src = blk_off[t], len = blk_off[t + 1] - src, dst = koff[t];
    if (threadIdx.x == 0) {
        new_col[d] = col_idx[t];
        new_off[d] = dst;
    }
    for (int64_t e = threadIdx.x; e < len; e += 64) new_vals[dst + e] = vals[src + e];
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

int compact_by_norm(Mat &m, const double *sq, const double *mx, double eps, int norm,
                    hipStream_t s, int64_t *nnzb_after, CompactKeep *keep) {
    const int64_t n = m.nnzb;
    *nnzb_after = n;
    if (n == 0) return BSM_OK;
    int64_t *kidx = nullptr, *koff = nullptr;
    BSM_TRY(dalloc(&kidx, n + 1, s));
    int st = dalloc(&koff, n + 1, s);
    if (st != BSM_OK) { dfree(kidx, s); return st; }
    k_keep<<<grid_for(n, 256), 256, 0, s>>>(sq, mx, m.blk_off, n, eps, norm, kidx, koff);
    st = scan_i64(kidx, kidx, n, s);
    if (st == BSM_OK) st = scan_i64(koff, koff, n, s);
    int64_t tot[2] = {0, 0};
    if (st == BSM_OK) {
        hipError_t e1 = hipMemcpyAsync(&tot[0], kidx + n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        hipError_t e2 = hipMemcpyAsync(&tot[1], koff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        hipError_t e3 = hipStreamSynchronize(s);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            set_error("filter: reading kept sizes failed");
            st = BSM_EDEVICE;
        }
    }
    if (st == BSM_OK && tot[0] != n) {
        Mat nm;
        st = dalloc(&nm.row_ptr, m.nbrows + 1, s);
        if (st == BSM_OK) st = dalloc(&nm.col_idx, tot[0], s);
        if (st == BSM_OK) st = dalloc(&nm.blk_off, tot[0] + 1, s);
        if (st == BSM_OK) st = dalloc(&nm.values, tot[1], s);
        if (st == BSM_OK) {
            k_compact_rows<<<grid_for(m.nbrows + 1, 256), 256, 0, s>>>(m.row_ptr, kidx, m.nbrows,
                                                                      nm.row_ptr);
            k_compact_blocks<<<static_cast<unsigned>(n), 64, 0, s>>>(
                kidx, koff, m.col_idx, m.blk_off, m.values, n, nm.col_idx, nm.blk_off, nm.values);
            k_set_i64<<<1, 1, 0, s>>>(nm.blk_off + tot[0], tot[1]);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) { set_error("filter kernels: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
        }
        if (st == BSM_OK) {
            if (keep) {
                keep->row_ptr = m.row_ptr; keep->col_idx = m.col_idx;
                keep->blk_off = m.blk_off; keep->values = m.values;
                keep->compacted = true;
            } else {
                free_mat_arrays(m, s);
            }
            m.row_ptr = nm.row_ptr; m.col_idx = nm.col_idx; m.blk_off = nm.blk_off;
            m.values = nm.values;
            m.nnzb = tot[0];
            m.nvalues = tot[1];
        } else {
            dfree(nm.row_ptr, s); dfree(nm.col_idx, s); dfree(nm.blk_off, s); dfree(nm.values, s);
        }
    }
    if (keep && st == BSM_OK) {
        keep->kidx = kidx;
        keep->koff = koff;
    } else {
        dfree(kidx, s);
        dfree(koff, s);
    }
    *nnzb_after = m.nnzb;
    return st;
}

int filter_inplace(Mat &m, double eps, int norm, hipStream_t s) {
    if (m.nnzb == 0 || eps == 0.0) return BSM_OK;
    double *sq = nullptr, *mx = nullptr;
    BSM_TRY(dalloc(&sq, m.nnzb, s));
    int st = dalloc(&mx, m.nnzb, s);
    if (st == BSM_OK) {
        k_block_norms<<<grid_for(m.nnzb, kRedThreads / kWave), kRedThreads, 0, s>>>(
            m.blk_off, m.values, m.nnzb, sq, mx);
        int64_t after = 0;
        st = compact_by_norm(m, sq, mx, eps, norm, s, &after);
    }
    dfree(sq, s);
    dfree(mx, s);
    return st;
}

// -------------------------------------------------------- row reductions

__device__ inline int64_t find_in_row(const int64_t *row_ptr, const int32_t *col_idx, int32_t i,
                                      int32_t j) {
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const int32_t c = col_idx[mid];
        if (c == j) return mid;
        if (c < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// Per block row: sum of the diagonal of the diagonal block.
__global__ void k_trace_rows(const int64_t *row_ptr, const int32_t *col_idx,
                             const int64_t *blk_off, const double *vals, const int32_t *rbs,
                             int32_t nbrows, double *part) {
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nbrows) return;
    const int64_t t = find_in_row(row_ptr, col_idx, i, i);
    double s = 0.0;
    if (t >= 0) {
        const int m = rbs[i];
        for (int r = 0; r < m; ++r) s += vals[blk_off[t] + r * m + r];
    }
    part[i] = s;
}

int trace(const Mat &m, double *out, hipStream_t s) {
    if (m.nbrows != m.nbcols) { set_error("trace needs a square block matrix"); return BSM_EINVAL; }
    *out = 0.0;
    if (m.nbrows == 0) return BSM_OK;
    double *part = nullptr;
    BSM_TRY(dalloc(&part, m.nbrows, s));
    k_trace_rows<<<grid_for(m.nbrows, 128), 128, 0, s>>>(m.row_ptr, m.col_idx, m.blk_off,
                                                        m.values, m.rbs, m.nbrows, part);
    int st = reduce_to_host(part, m.nbrows, 0, out, s);
    dfree(part, s);
    return st;
}

// Per block row: sum over its blocks of (x - shift*delta)^2, plus
// m*shift^2 when the diagonal block is missing.  Waves take blocks in turn;
// the per-wave sums are added in wave order.
__global__ void __launch_bounds__(kRedThreads)
k_sqdist_rows(const int64_t *row_ptr, const int32_t *col_idx, const int64_t *blk_off,
              const double *vals, const int32_t *rbs, const int32_t *cbs, double shift,
              double *part) {
    __shared__ double wpart[kRedThreads / kWave];
    __shared__ int has_diag;
    const int32_t i = blockIdx.x;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (threadIdx.x == 0) has_diag = 0;
    __syncthreads();
    const int m = rbs[i];
    double acc = 0.0;
    for (int64_t t = row_ptr[i] + wid; t < row_ptr[i + 1]; t += kRedThreads / kWave) {
        const int32_t j = col_idx[t];
        const int n = cbs[j];
        const double *x = vals + blk_off[t];
        double s = 0.0;
        for (int e = lane; e < m * n; e += kWave) {
            double v = x[e];
            if (j == i && (e / n) == (e % n)) v -= shift;
            s += v * v;
        }
        acc += s;
        if (j == i && lane == 0) has_diag = 1;
    }
    acc = wsum(acc);
    if (lane == 0) wpart[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < kRedThreads / kWave; ++w) r += wpart[w];
        if (!has_diag) r += static_cast<double>(m) * shift * shift;
        part[i] = r;
    }
}

int sqdist_identity_dev(const Mat &m, double shift, double *part, double *d_out, hipStream_t s) {
    if (m.nbrows == 0) { set_error("empty matrix"); return BSM_EINVAL; }
    k_sqdist_rows<<<m.nbrows, kRedThreads, 0, s>>>(m.row_ptr, m.col_idx, m.blk_off, m.values,
                                                   m.rbs, m.cbs, shift, part);
    k_reduce_final<<<1, 1024, 0, s>>>(part, m.nbrows, d_out, 0);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

__global__ void k_set_f64(double *p, double v) { *p = v; }

int sqdist_identity_noalloc(const Mat &m, double shift, double *out_dev, hipStream_t s) {
    if (m.nbrows != m.nbcols) { set_error("needs a square block matrix"); return BSM_EINVAL; }
    if (m.nbrows > kNoAllocMaxRows) {
        set_error("%d block rows exceed the fixed scratch of %lld rows", m.nbrows,
                  static_cast<long long>(kNoAllocMaxRows));
        return BSM_ECAPACITY;
    }
    int dev = 0;
    BSM_HIP(hipGetDevice(&dev));
    if (dev != m.device) {
        set_error("the matrix lives on device %d, device %d is current", m.device, dev);
        return BSM_EINVAL;
    }
    if (m.nbrows == 0) {
        k_set_f64<<<1, 1, 0, s>>>(out_dev, 0.0);
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
    double *part = nullptr;
    BSM_TRY(scratch_address(&part));
    k_sqdist_rows<<<m.nbrows, kRedThreads, 0, s>>>(m.row_ptr, m.col_idx, m.blk_off, m.values,
                                                   m.rbs, m.cbs, shift, part);
    k_reduce_final<<<1, 1024, 0, s>>>(part, m.nbrows, out_dev, 0);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int sqdist_identity(const Mat &m, double shift, double *out, hipStream_t s) {
    if (m.nbrows != m.nbcols) { set_error("needs a square block matrix"); return BSM_EINVAL; }
    *out = 0.0;
    if (m.nbrows == 0) return BSM_OK;
    double *part = nullptr;
    BSM_TRY(dalloc(&part, m.nbrows, s));
    k_sqdist_rows<<<m.nbrows, kRedThreads, 0, s>>>(m.row_ptr, m.col_idx, m.blk_off, m.values,
                                                   m.rbs, m.cbs, shift, part);
    int st = reduce_to_host(part, m.nbrows, 0, out, s);
    dfree(part, s);
    return st;
}

// Per block row: the largest scalar-row sum of |(A - mu I)_rc|.  Lane r
// (r < 32) walks even blocks, lane r + 32 odd blocks; the halves are added.
__global__ void __launch_bounds__(64)
k_inf_rows(const int64_t *row_ptr, const int32_t *col_idx, const int64_t *blk_off,
           const double *vals, const int32_t *rbs, const int32_t *cbs, double mu, double *part) {
    const int32_t i = blockIdx.x;
    const int lane = threadIdx.x, r = lane & 31, half = lane >> 5;
    const int m = rbs[i];
    double s = 0.0;
    int seen_diag = 0;
    if (r < m) {
        for (int64_t t = row_ptr[i] + half; t < row_ptr[i + 1]; t += 2) {
            const int32_t j = col_idx[t];
            const int n = cbs[j];
            const double *x = vals + blk_off[t] + static_cast<int64_t>(r) * n;
            for (int c = 0; c < n; ++c) s += fabs(x[c] - ((j == i && c == r) ? mu : 0.0));
            if (j == i) seen_diag = 1;
        }
    }
    const double other = __shfl_down(s, 32, kWave);
    const int other_diag = __shfl_down(seen_diag, 32, kWave);
    double rowsum = s + other;
    if (!(seen_diag | other_diag)) rowsum += fabs(mu);
    double v = (half == 0 && r < m) ? rowsum : 0.0;
    v = wmax(v);
    if (lane == 0) part[i] = v;
}

int inf_norm(const Mat &m, double mu, double *out, hipStream_t s) {
    *out = 0.0;
    if (m.nbrows == 0) return BSM_OK;
    if (m.nbrows != m.nbcols && mu != 0.0) { set_error("shifted norm needs a square matrix"); return BSM_EINVAL; }
    double *part = nullptr;
    BSM_TRY(dalloc(&part, m.nbrows, s));
    k_inf_rows<<<m.nbrows, 64, 0, s>>>(m.row_ptr, m.col_idx, m.blk_off, m.values, m.rbs, m.cbs,
                                       mu, part);
    int st = reduce_to_host(part, m.nbrows, 1, out, s);
    dfree(part, s);
    return st;
}

// ---------------------------------------------------- shift, scale, copy

__global__ void k_diag_missing(const int64_t *row_ptr, const int32_t *col_idx, int32_t nbrows,
                               int64_t *miss) {
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nbrows) return;
    miss[i] = find_in_row(row_ptr, col_idx, i, i) < 0 ? 1 : 0;
}

// New pattern: old pattern plus the missing diagonal blocks.
__global__ void k_diag_insert_pattern(const int64_t *row_ptr, const int32_t *col_idx,
                                      const int64_t *miss_scan, int32_t nbrows,
                                      int64_t *new_row_ptr, int32_t *new_col, int64_t *src) {
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i > nbrows) return;
    const int64_t base = row_ptr[i] + miss_scan[i];
    new_row_ptr[i] = base;
    if (i == nbrows) return;
    const bool ins = (miss_scan[i + 1] - miss_scan[i]) != 0;
    int64_t d = base;
    bool done = !ins;
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
        if (!done && col_idx[t] > i) { new_col[d] = i; src[d] = -1; ++d; done = true; }
        new_col[d] = col_idx[t]; src[d] = t; ++d;
    }
    if (!done) { new_col[d] = i; src[d] = -1; }
}

// One workgroup per new block: out = scale * (x - mu * delta).
__global__ void __launch_bounds__(64)
k_shift_scale_vals(const int64_t *new_row_ptr, const int32_t *new_col, const int64_t *src,
                   const int64_t *new_off, const int64_t *old_off, const double *old_vals,
                   const int32_t *rbs, const int32_t *cbs, int32_t nbrows, double mu, double scale,
                   double *out) {
    const int64_t d = blockIdx.x;
    // block row of d by binary search over new_row_ptr
    int32_t lo = 0, hi = nbrows - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (new_row_ptr[mid] <= d) lo = mid; else hi = mid - 1;
    }
    const int32_t i = lo, j = new_col[d];
    const int m = rbs[i], n = cbs[j];
    const int64_t so = src[d];
    for (int e = threadIdx.x; e < m * n; e += 64) {
        const double x = so >= 0 ? old_vals[old_off[so] + e] : 0.0;
        const double sh = (i == j && (e / n) == (e % n)) ? mu : 0.0;
        out[new_off[d] + e] = scale * (x - sh);
    }
}

int new_mat_sizes(const Mat &r, bool r_cols, const Mat &c, bool c_rows, Mat **out, hipStream_t s) {
    Mat *m = new Mat;
    m->device = r.device;
    m->nbrows = r_cols ? r.nbcols : r.nbrows;
    m->nrows = r_cols ? r.ncols : r.nrows;
    m->h_rbs = r_cols ? r.h_cbs : r.h_rbs;
    m->max_rbs = r_cols ? r.max_cbs : r.max_rbs;
    m->uni_r = r_cols ? r.uni_c : r.uni_r;
    m->nbcols = c_rows ? c.nbrows : c.nbcols;
    m->ncols = c_rows ? c.nrows : c.ncols;
    m->h_cbs = c_rows ? c.h_rbs : c.h_cbs;
    m->max_cbs = c_rows ? c.max_rbs : c.max_cbs;
    m->uni_c = c_rows ? c.uni_r : c.uni_c;
    const int32_t *rsz = r_cols ? r.cbs : r.rbs;
    const int64_t *rof = r_cols ? r.coff : r.roff;
    const int32_t *csz = c_rows ? c.rbs : c.cbs;
    const int64_t *cof = c_rows ? c.roff : c.coff;
    int st = dalloc(&m->rbs, m->nbrows, s);
    if (st == BSM_OK) st = dalloc(&m->cbs, m->nbcols, s);
    if (st == BSM_OK) st = dalloc(&m->roff, m->nbrows + 1, s);
    if (st == BSM_OK) st = dalloc(&m->coff, m->nbcols + 1, s);
    if (st == BSM_OK) {
        hipError_t e = hipMemcpyAsync(m->rbs, rsz, sizeof(int32_t) * m->nbrows, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(m->cbs, csz, sizeof(int32_t) * m->nbcols, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(m->roff, rof, sizeof(int64_t) * (m->nbrows + 1), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(m->coff, cof, sizeof(int64_t) * (m->nbcols + 1), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) { set_error("copy of block sizes failed: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st != BSM_OK) { free_mat(m, s); return st; }
    m->stream = s;
    *out = m;
    return BSM_OK;
}

static int new_mat_like(const Mat &a, Mat **out, hipStream_t s) {
    return new_mat_sizes(a, false, a, false, out, s);
}

int alloc_like_sizes(const Mat &rows, const Mat &cols, Mat **out, hipStream_t s) {
    return new_mat_sizes(rows, false, cols, false, out, s);
}

int shift_scale(const Mat &a, double mu, double scale, Mat **out, hipStream_t s) {
    if (a.nbrows != a.nbcols) { set_error("shift needs a square block matrix"); return BSM_EINVAL; }
    for (int32_t i = 0; i < a.nbrows; ++i)
        if (a.h_rbs[i] != a.h_cbs[i]) { set_error("shift needs square diagonal blocks"); return BSM_EINVAL; }
    Mat *m = nullptr;
    BSM_TRY(new_mat_like(a, &m, s));
    int64_t *miss = nullptr, *src = nullptr;
    int st = dalloc(&miss, a.nbrows + 1, s);
    int64_t nmiss = 0;
    if (st == BSM_OK && a.nbrows > 0) {
        k_diag_missing<<<grid_for(a.nbrows, 128), 128, 0, s>>>(a.row_ptr, a.col_idx, a.nbrows, miss);
        st = scan_i64(miss, miss, a.nbrows, s);
        if (st == BSM_OK) {
            hipError_t e = hipMemcpyAsync(&nmiss, miss + a.nbrows, sizeof(int64_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { set_error("shift: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
        }
    }
    const int64_t nnzb = a.nnzb + nmiss;
    if (st == BSM_OK) st = dalloc(&m->row_ptr, a.nbrows + 1, s);
    if (st == BSM_OK) st = dalloc(&m->col_idx, nnzb, s);
    if (st == BSM_OK) st = dalloc(&src, nnzb, s);
    if (st == BSM_OK) {
        if (a.nbrows > 0) {
            k_diag_insert_pattern<<<grid_for(a.nbrows + 1, 128), 128, 0, s>>>(
                a.row_ptr, a.col_idx, miss, a.nbrows, m->row_ptr, m->col_idx, src);
        } else {
            hipError_t e = hipMemsetAsync(m->row_ptr, 0, sizeof(int64_t), s);
            if (e != hipSuccess) st = BSM_EDEVICE;
        }
        m->nnzb = nnzb;
    }
    if (st == BSM_OK) st = compute_blk_off(*m, s);
    if (st == BSM_OK) {
        int64_t nv = 0;
        hipError_t e = hipMemcpyAsync(&nv, m->blk_off + nnzb, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { set_error("shift: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
        m->nvalues = nv;
        if (st == BSM_OK) st = dalloc(&m->values, nv, s);
    }
    if (st == BSM_OK && nnzb > 0) {
        k_shift_scale_vals<<<static_cast<unsigned>(nnzb), 64, 0, s>>>(
            m->row_ptr, m->col_idx, src, m->blk_off, a.blk_off, a.values, a.rbs, a.cbs, a.nbrows,
            mu, scale, m->values);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_error("shift kernel: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    dfree(miss, s);
    dfree(src, s);
    if (st != BSM_OK) { free_mat(m, s); return st; }
    *out = m;
    return BSM_OK;
}

int copy_mat(const Mat &a, Mat **out, hipStream_t s) {
    Mat *m = nullptr;
    BSM_TRY(new_mat_like(a, &m, s));
    m->nnzb = a.nnzb;
    m->nvalues = a.nvalues;
    int st = dalloc(&m->row_ptr, a.nbrows + 1, s);
    if (st == BSM_OK) st = dalloc(&m->col_idx, a.nnzb, s);
    if (st == BSM_OK) st = dalloc(&m->blk_off, a.nnzb + 1, s);
    if (st == BSM_OK) st = dalloc(&m->values, a.nvalues, s);
    if (st == BSM_OK) {
        hipError_t e = hipMemcpyAsync(m->row_ptr, a.row_ptr, sizeof(int64_t) * (a.nbrows + 1), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && a.nnzb) e = hipMemcpyAsync(m->col_idx, a.col_idx, sizeof(int32_t) * a.nnzb, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(m->blk_off, a.blk_off, sizeof(int64_t) * (a.nnzb + 1), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && a.nvalues) e = hipMemcpyAsync(m->values, a.values, sizeof(double) * a.nvalues, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) { set_error("copy: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st != BSM_OK) { free_mat(m, s); return st; }
    *out = m;
    return BSM_OK;
}

}  // namespace bsm
