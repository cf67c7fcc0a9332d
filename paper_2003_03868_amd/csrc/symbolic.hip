// Symbolic phase of the block-sparse multiply: which blocks of C exist and
// which block products feed each of them.  This is the "what will be
// multiplied" half of the DBCSR local multiply (Local multiplication
// subsection: traversal over A block rows, then batches of block products),
// done on the device.  The numeric half (smm.hip) then only executes stacks.
//
// One workgroup owns one block row i of C.  It marks the block columns j
// reached through A_ik B_kj (and C_in's row when beta != 0) in an LDS bitmap
// of nbcols bits; the rank of j among the marked bits is its position in C's
// row.  Product stacks are C-stationary: the products of block (i,j) form one
// contiguous segment ordered by ascending k, so one wavefront later owns the
// whole C block and sums in a fixed order without atomics.
#include "symbolic.h"

namespace bsm {

constexpr int kSymThreads = 256;
constexpr int kSymWaves = kSymThreads / kWave;

__device__ inline void mark_row_bits(uint32_t *bits, const SymArgs &a, int32_t i) {
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    for (int64_t ta = a.a_row_ptr[i] + wid; ta < a.a_row_ptr[i + 1]; ta += kSymWaves) {
        const int32_t k = a.a_col_idx[ta];
        for (int64_t tb = a.b_row_ptr[k] + lane; tb < a.b_row_ptr[k + 1]; tb += kWave) {
            const int32_t j = a.b_col_idx[tb];
            atomicOr(&bits[j >> 5], 1u << (j & 31));
        }
    }
    if (a.use_c) {
        for (int64_t tc = a.c_in_row_ptr[i] + threadIdx.x; tc < a.c_in_row_ptr[i + 1];
             tc += kSymThreads) {
            const int32_t j = a.c_in_col_idx[tc];
            atomicOr(&bits[j >> 5], 1u << (j & 31));
        }
    }
}

// Sum over the workgroup (fixed order: wave shuffles, then waves in order).
template <class T>
__device__ inline T wg_sum(T v, T *scratch) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < kSymWaves; ++w) s += scratch[w];
    __syncthreads();
    return s;
}

// Workgroup exclusive scan of one value per thread; *total gets the sum.
template <class T>
__device__ inline T wg_exscan(T v, T *scratch, T *total) {
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    T x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) scratch[wid] = x;
    __syncthreads();
    T before = 0, all = 0;
    for (int w = 0; w < kSymWaves; ++w) {
        if (w < wid) before += scratch[w];
        all += scratch[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Per C block row: number of C blocks, stored C scalars, block products and
// their flops (2 m n k each).
__global__ void __launch_bounds__(kSymThreads)
k_sym_count(SymArgs a, int64_t *c_cnt, int64_t *c_nval, int64_t *p_cnt, double *flops) {
    extern __shared__ uint32_t bits[];
    __shared__ int64_t red_i[kSymWaves];
    __shared__ double red_d[kSymWaves];
    const int32_t i = blockIdx.x;
    const int nwords = (a.nbcols + 31) >> 5;
    for (int w = threadIdx.x; w < nwords; w += kSymThreads) bits[w] = 0u;
    __syncthreads();
    mark_row_bits(bits, a, i);

    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int64_t m = a.c_rbs[i];
    int64_t prods = 0;
    double fl = 0.0;
    for (int64_t ta = a.a_row_ptr[i] + wid; ta < a.a_row_ptr[i + 1]; ta += kSymWaves) {
        const int32_t k = a.a_col_idx[ta];
        const int64_t kk = a.k_size[k];
        for (int64_t tb = a.b_row_ptr[k] + lane; tb < a.b_row_ptr[k + 1]; tb += kWave) {
            prods += 1;
            fl += 2.0 * static_cast<double>(m * kk * a.c_cbs[a.b_col_idx[tb]]);
        }
    }
    __syncthreads();
    int64_t nblk = 0, nval = 0;
    for (int w = threadIdx.x; w < nwords; w += kSymThreads) {
        uint32_t x = bits[w];
        nblk += __popc(x);
        while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1;
            nval += m * a.c_cbs[w * 32 + b];
        }
    }
    nblk = wg_sum(nblk, red_i);
    nval = wg_sum(nval, red_i);
    prods = wg_sum(prods, red_i);
    fl = wg_sum(fl, red_d);
    if (threadIdx.x == 0) {
        c_cnt[i] = nblk;
        c_nval[i] = nval;
        p_cnt[i] = prods;
        flops[i] = fl;
    }
}

// Rank of column j among the marked bits of the row.
__device__ inline int32_t bit_rank(const uint32_t *bits, const int32_t *wpre, int32_t j) {
    const uint32_t w = bits[j >> 5];
    const uint32_t below = (j & 31) ? (w & ((1u << (j & 31)) - 1u)) : 0u;
    return wpre[j >> 5] + __popc(below);
}

// Builds bitmap + exclusive popcount prefix per word in LDS.
__device__ inline void build_rank(uint32_t *bits, int32_t *wpre, const SymArgs &a, int32_t i,
                                  int32_t *scratch) {
    const int nwords = (a.nbcols + 31) >> 5;
    for (int w = threadIdx.x; w < nwords; w += kSymThreads) bits[w] = 0u;
    __syncthreads();
    mark_row_bits(bits, a, i);
    __syncthreads();
    const int per = (nwords + kSymThreads - 1) / kSymThreads;
    const int w0 = threadIdx.x * per;
    int32_t local = 0;
    for (int w = w0; w < w0 + per && w < nwords; ++w) local += __popc(bits[w]);
    int32_t total;
    int32_t run = wg_exscan(local, scratch, &total);
    for (int w = w0; w < w0 + per && w < nwords; ++w) {
        wpre[w] = run;
        run += __popc(bits[w]);
    }
    __syncthreads();
}

// C pattern: col_idx, owning row, and the matching C_in block (or -1).
__global__ void __launch_bounds__(kSymThreads)
k_sym_pattern(SymArgs a, const int64_t *c_row_ptr, int32_t *c_col_idx, int32_t *c_row,
              int64_t *cin_map) {
    extern __shared__ uint32_t smem[];
    __shared__ int32_t scratch[kSymWaves];
    const int nwords = (a.nbcols + 31) >> 5;
    uint32_t *bits = smem;
    int32_t *wpre = reinterpret_cast<int32_t *>(smem + nwords);
    const int32_t i = blockIdx.x;
    build_rank(bits, wpre, a, i, scratch);
    // writes stay inside the row's range of c_row_ptr (all of the row's
    // blocks when the counts came from k_sym_count; none when a caller
    // emptied the rows after a capacity overflow)
    const int64_t base = c_row_ptr[i], end = c_row_ptr[i + 1];
    for (int w = threadIdx.x; w < nwords; w += kSymThreads) {
        uint32_t x = bits[w];
        int32_t r = wpre[w];
        while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1;
            if (base + r < end) {
                c_col_idx[base + r] = w * 32 + b;
                c_row[base + r] = i;
                if (cin_map) cin_map[base + r] = -1;
            }
            ++r;
        }
    }
    if (a.use_c && cin_map) {
        __syncthreads();
        for (int64_t tc = a.c_in_row_ptr[i] + threadIdx.x; tc < a.c_in_row_ptr[i + 1];
             tc += kSymThreads) {
            const int64_t pos = base + bit_rank(bits, wpre, a.c_in_col_idx[tc]);
            if (pos < end) cin_map[pos] = tc;
        }
    }
}

// Product stacks for the block rows [r0, r0 + gridDim.x): per C block the
// segment [seg[c-c0], seg[c-c0+1]) of (a block, b block) pairs, ascending k.
// Positions are relative to the first product of row r0 (p_base).
__global__ void __launch_bounds__(kSymThreads)
k_sym_stack(SymArgs a, int32_t r0, int32_t r1, const int64_t *c_row_ptr,
            const int64_t *p_row_ptr, int64_t *seg, int32_t *stk_a, int32_t *stk_b) {
    extern __shared__ uint32_t smem[];
    __shared__ int32_t scratch[kSymWaves];
    __shared__ int64_t scratch64[kSymWaves];
    const int nwords = (a.nbcols + 31) >> 5;
    uint32_t *bits = smem;
    int32_t *wpre = reinterpret_cast<int32_t *>(smem + nwords);
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + 2 * nwords);
    const int32_t i = r0 + blockIdx.x;
    build_rank(bits, wpre, a, i, scratch);

    const int64_t c0 = c_row_ptr[r0];
    const int64_t cb = c_row_ptr[i], nrow = c_row_ptr[i + 1] - cb;
    const int64_t p_base = p_row_ptr[r0];
    int64_t carry = p_row_ptr[i] - p_base;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int64_t a_beg = a.a_row_ptr[i], a_end = a.a_row_ptr[i + 1];

    for (int64_t w0 = 0; w0 < nrow; w0 += kStackWindow) {
        const int wn = static_cast<int>(nrow - w0 < kStackWindow ? nrow - w0 : kStackWindow);
        for (int q = threadIdx.x; q < wn; q += kSymThreads) cnt[q] = 0;
        __syncthreads();
        // count products per C block of the window
        for (int64_t ta = a_beg + wid; ta < a_end; ta += kSymWaves) {
            const int32_t k = a.a_col_idx[ta];
            for (int64_t tb = a.b_row_ptr[k] + lane; tb < a.b_row_ptr[k + 1]; tb += kWave) {
                const int64_t r = bit_rank(bits, wpre, a.b_col_idx[tb]) - w0;
                if (r >= 0 && r < wn) atomicAdd(&cnt[r], 1);
            }
        }
        __syncthreads();
        // exclusive scan of the window counts -> segment starts (cursors)
        const int per = (wn + kSymThreads - 1) / kSymThreads;
        const int q0 = threadIdx.x * per;
        int64_t local = 0;
        for (int q = q0; q < q0 + per && q < wn; ++q) local += cnt[q];
        int64_t total;
        int64_t run = wg_exscan(local, scratch64, &total) + carry;
        for (int q = q0; q < q0 + per && q < wn; ++q) {
            const int32_t cq = cnt[q];
            seg[cb + w0 + q - c0] = run;
            cnt[q] = static_cast<int32_t>(run - carry);   // cursor relative to carry
            run += cq;
        }
        __syncthreads();
        // fill, one A block at a time so each segment stays in ascending k
        for (int64_t ta = a_beg; ta < a_end; ++ta) {
            const int32_t k = a.a_col_idx[ta];
            for (int64_t tb = a.b_row_ptr[k] + threadIdx.x; tb < a.b_row_ptr[k + 1];
                 tb += kSymThreads) {
                const int64_t r = bit_rank(bits, wpre, a.b_col_idx[tb]) - w0;
                if (r >= 0 && r < wn) {
                    const int64_t pos = carry + cnt[r];
                    cnt[r] += 1;
                    stk_a[pos] = static_cast<int32_t>(ta);
                    stk_b[pos] = static_cast<int32_t>(tb);
                }
            }
            __syncthreads();
        }
        carry += total;
    }
    if (i == r1 - 1 && threadIdx.x == 0) seg[c_row_ptr[r1] - c0] = p_row_ptr[r1] - p_base;
}

// Tiled work order of the C blocks of one band of `rb` block rows: C blocks
// are grouped by column band (`wb` consecutive block columns), then by row,
// then by column.  Waves that run together on one XCD then share A blocks
// (same row) and B blocks (same column) in that XCD's L2.  worklist[pos] =
// C block index, pos covering the band's C blocks in the new order.
constexpr int kOrderMaxRows = 16;
constexpr int kOrderMaxBands = 256;

__global__ void __launch_bounds__(kSymThreads)
k_tile_order(const int64_t *c_row_ptr, const int32_t *c_col_idx, int32_t nbrows, int rb, int wb,
             int nbands, int64_t *worklist) {
    __shared__ int32_t cnt[kOrderMaxRows * kOrderMaxBands];    // [row][band]
    __shared__ int32_t start[kOrderMaxRows * kOrderMaxBands];  // position in band order
    __shared__ int32_t rowpre[kOrderMaxRows * kOrderMaxBands]; // CSR offset in the row
    __shared__ int32_t scratch[kSymWaves];
    const int32_t i0 = blockIdx.x * rb;
    const int32_t i1 = min(i0 + rb, nbrows);
    const int nr = i1 - i0;
    const int cells = nr * nbands;
    for (int q = threadIdx.x; q < cells; q += kSymThreads) cnt[q] = 0;
    __syncthreads();
    const int64_t cb0 = c_row_ptr[i0];
    for (int r = 0; r < nr; ++r)
        for (int64_t c = c_row_ptr[i0 + r] + threadIdx.x; c < c_row_ptr[i0 + r + 1];
             c += kSymThreads)
            atomicAdd(&cnt[r * nbands + c_col_idx[c] / wb], 1);
    __syncthreads();
    // exclusive scan in (band, row) order -> start; along bands per row -> rowpre
    const int per = (cells + kSymThreads - 1) / kSymThreads;
    const int q0 = threadIdx.x * per;
    int32_t local = 0;
    for (int q = q0; q < q0 + per && q < cells; ++q) {
        const int band = q / nr, r = q % nr;
        local += cnt[r * nbands + band];
    }
    int32_t total;
    int32_t run = wg_exscan(local, scratch, &total);
    for (int q = q0; q < q0 + per && q < cells; ++q) {
        const int band = q / nr, r = q % nr;
        start[r * nbands + band] = run;
        run += cnt[r * nbands + band];
    }
    if (threadIdx.x < nr) {
        int32_t acc = 0;
        for (int band = 0; band < nbands; ++band) {
            rowpre[threadIdx.x * nbands + band] = acc;
            acc += cnt[threadIdx.x * nbands + band];
        }
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
        const int64_t rs = c_row_ptr[i0 + r];
        for (int64_t c = rs + threadIdx.x; c < c_row_ptr[i0 + r + 1]; c += kSymThreads) {
            const int band = c_col_idx[c] / wb;
            const int64_t pos = start[r * nbands + band] + (c - rs - rowpre[r * nbands + band]);
            worklist[cb0 + pos] = c;
        }
    }
}

int tile_order(const int64_t *c_row_ptr, const int32_t *c_col_idx, int32_t nbrows,
               int32_t nbcols, int rb, int64_t *worklist, hipStream_t s, int wb) {
    if (nbrows == 0) return BSM_OK;
    if (rb < 1 || rb > kOrderMaxRows) { set_error("tile rows must be in [1, %d]", kOrderMaxRows); return BSM_EINVAL; }
    if (wb < 1) wb = tile_cols();
    if ((nbcols + wb - 1) / wb > kOrderMaxBands) wb = (nbcols + kOrderMaxBands - 1) / kOrderMaxBands;
    const int nbands = (nbcols + wb - 1) / wb;
    const int nb = (nbrows + rb - 1) / rb;
    k_tile_order<<<nb, kSymThreads, 0, s>>>(c_row_ptr, c_col_idx, nbrows, rb, wb, nbands,
                                            worklist);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// ---------------------------------------------------------- work-list sort
// Bucket sort of a chunk's work list (the paper sorts stacks by (m, n, k) so
// that homogeneous batches reach specialised kernels).  Key modes:
//   kKeyCost:  bucket = 63 - floor(log2(cost)), cost = products * m * n, so
//              ascending buckets are descending cost (largest stacks first);
//   kKeyClass: bucket = 4*class(m) + class(n) for sizes {5,13,23,26}, 16 else.
// Within a bucket the order is that of the input list within a workgroup.
constexpr int kSortThreads = 256;
constexpr int kMaxBuckets = 64;

__device__ inline int class_of(int b) { return b == 5 ? 0 : b == 13 ? 1 : b == 23 ? 2 : b == 26 ? 3 : -1; }

__device__ inline int wl_key(int mode, int64_t c, int64_t c0, const int32_t *c_row,
                             const int32_t *c_col, const int32_t *rbs, const int32_t *cbs,
                             const int64_t *seg) {
    const int m = rbs[c_row[c]], n = cbs[c_col[c]];
    if (mode == kKeyClass) {
        const int cm = class_of(m), cn = class_of(n);
        return (cm < 0 || cn < 0) ? 16 : 4 * cm + cn;
    }
    const unsigned long long cost =
        static_cast<unsigned long long>(seg[c - c0 + 1] - seg[c - c0]) * m * n + 1ull;
    const int lg = 63 - __clzll(cost);
    return 63 - lg;
}

__global__ void __launch_bounds__(kSortThreads)
k_wl_hist(const int64_t *wl, int64_t n, int64_t c0, int mode, const int32_t *c_row,
          const int32_t *c_col, const int32_t *rbs, const int32_t *cbs, const int64_t *seg,
          unsigned long long *hist) {
    __shared__ unsigned int lh[kMaxBuckets];
    if (threadIdx.x < kMaxBuckets) lh[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&lh[wl_key(mode, wl[c0 + i], c0, c_row, c_col, rbs, cbs, seg)], 1u);
    __syncthreads();
    if (threadIdx.x < kMaxBuckets && lh[threadIdx.x])
        atomicAdd(&hist[threadIdx.x], static_cast<unsigned long long>(lh[threadIdx.x]));
}

// cursor[b] starts at the bucket's first position; each workgroup reserves
// one range per bucket and places its elements in thread order.
__global__ void __launch_bounds__(kSortThreads)
k_wl_scatter(const int64_t *wl, int64_t n, int64_t c0, int mode, const int32_t *c_row,
             const int32_t *c_col, const int32_t *rbs, const int32_t *cbs, const int64_t *seg,
             unsigned long long *cursor, int64_t *out) {
    __shared__ unsigned int lh[kMaxBuckets];
    __shared__ unsigned long long base[kMaxBuckets];
    __shared__ int keys[kSortThreads];
    if (threadIdx.x < kMaxBuckets) lh[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kSortThreads + threadIdx.x;
    int key = -1;
    int64_t c = 0;
    if (i < n) {
        c = wl[c0 + i];
        key = wl_key(mode, c, c0, c_row, c_col, rbs, cbs, seg);
        atomicAdd(&lh[key], 1u);
    }
    keys[threadIdx.x] = key;
    __syncthreads();
    if (threadIdx.x < kMaxBuckets && lh[threadIdx.x])
        base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], static_cast<unsigned long long>(lh[threadIdx.x]));
    __syncthreads();
    if (key >= 0) {
        unsigned int rank = 0;
        for (int t = 0; t < static_cast<int>(threadIdx.x); ++t) rank += (keys[t] == key);
        out[c0 + base[key] + rank] = c;
    }
}

__global__ void k_wl_zero(unsigned long long *p) { p[threadIdx.x] = 0ull; }

__global__ void k_wl_cursor(const unsigned long long *hist, unsigned long long *cursor) {
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (int b = 0; b < kMaxBuckets; ++b) { cursor[b] = run; run += hist[b]; }
    }
}

int sort_worklist(const int64_t *wl_in, int64_t *wl_out, int64_t c0, int64_t n, int mode,
                  const int32_t *c_row, const int32_t *c_col, const int32_t *rbs,
                  const int32_t *cbs, const int64_t *seg, int64_t *hist_host, hipStream_t s) {
    if (n <= 0) return BSM_OK;
    unsigned long long *buf = nullptr;
    BSM_TRY(dalloc(&buf, 2 * kMaxBuckets, s));
    unsigned long long *hist = buf, *cursor = buf + kMaxBuckets;
    k_wl_zero<<<1, 2 * kMaxBuckets, 0, s>>>(buf);
    const unsigned g = grid_for(n, kSortThreads);
    k_wl_hist<<<g, kSortThreads, 0, s>>>(wl_in, n, c0, mode, c_row, c_col, rbs, cbs, seg, hist);
    k_wl_cursor<<<1, 64, 0, s>>>(hist, cursor);
    k_wl_scatter<<<g, kSortThreads, 0, s>>>(wl_in, n, c0, mode, c_row, c_col, rbs, cbs, seg,
                                            cursor, wl_out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && hist_host) {
        unsigned long long h[kMaxBuckets];
        e = hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        for (int b = 0; b < kMaxBuckets; ++b) hist_host[b] = static_cast<int64_t>(h[b]);
    }
    dfree(buf, s);
    if (e != hipSuccess) { set_error("work-list sort: %s", hipGetErrorString(e)); return BSM_EDEVICE; }
    return BSM_OK;
}

int tile_rows() {
    const char *e = getenv("BSM_TILE_ROWS");
    const int v = e ? atoi(e) : 16;
    return v < 1 ? 1 : (v > kOrderMaxRows ? kOrderMaxRows : v);
}
int tile_cols() {
    const char *e = getenv("BSM_TILE_COLS");
    const int v = e ? atoi(e) : 32;
    return v < 1 ? 1 : v;
}

int sym_count(const SymArgs &a, int64_t *c_cnt, int64_t *c_nval, int64_t *p_cnt, double *flops,
              hipStream_t s) {
    if (a.nbrows == 0) return BSM_OK;
    const size_t lds = sizeof(uint32_t) * ((a.nbcols + 31) / 32);
    k_sym_count<<<a.nbrows, kSymThreads, lds, s>>>(a, c_cnt, c_nval, p_cnt, flops);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int sym_pattern(const SymArgs &a, const int64_t *c_row_ptr, int32_t *c_col_idx, int32_t *c_row,
                int64_t *cin_map, hipStream_t s) {
    if (a.nbrows == 0) return BSM_OK;
    const size_t lds = 2 * sizeof(uint32_t) * ((a.nbcols + 31) / 32);
    k_sym_pattern<<<a.nbrows, kSymThreads, lds, s>>>(a, c_row_ptr, c_col_idx, c_row, cin_map);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int sym_stack(const SymArgs &a, int32_t r0, int32_t r1, const int64_t *c_row_ptr,
              const int64_t *p_row_ptr, int64_t *seg, int32_t *stk_a, int32_t *stk_b,
              hipStream_t s) {
    if (r1 <= r0) return BSM_OK;
    const size_t lds = 2 * sizeof(uint32_t) * ((a.nbcols + 31) / 32) +
                       sizeof(int32_t) * kStackWindow;
    k_sym_stack<<<r1 - r0, kSymThreads, lds, s>>>(a, r0, r1, c_row_ptr, p_row_ptr, seg, stk_a,
                                                  stk_b);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
