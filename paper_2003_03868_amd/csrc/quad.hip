// Quads: 2 x 2 groups of C blocks with merged product lists (symbolic part
// of the quad block-product kernel in smm_quad.hip).  Built straight from
// the patterns of A, B and C, without per-C-block stacks.
//
// A quad is the group C(2R + r, 2Q + c), r, c in {0, 1}, of the C blocks of a
// chunk (at least one of them present).  Its entry list is the union of the
// k's of its C blocks' products, ascending; entry k names A(2R + r, k) for
// each row r and B(k, 2Q + c) for each column c that a product of the quad
// uses, -1 otherwise.  Product (r, c) of an entry exists exactly when both
// A(2R + r, k) and B(k, 2Q + c) are named, so the per-C-block sums are those
// of the plain stacks, in the same (ascending k) order, while every operand
// block is loaded once for up to four products.
#include <climits>

#include "symbolic.h"

namespace bsm {

constexpr int kQuadThreads = 256;

// Rank of column pair Q among the marked bits.
__device__ inline int32_t bit_rank_q(const uint32_t *bits, const int32_t *wpre, int32_t Q) {
    const uint32_t w = bits[Q >> 5];
    const uint32_t below = (Q & 31) ? (w & ((1u << (Q & 31)) - 1u)) : 0u;
    return wpre[Q >> 5] + __popc(below);
}

// ---------------------------------------------------------------------------
// Entry lists straight from the patterns of A and B: one workgroup per row
// pair walks k over the merged column lists of A's rows 2R and 2R + 1
// (ascending); for each k its threads scan B's row k, and the thread holding
// column j = 2Q (or 2Q + 1 when 2Q is absent) emits the entry of quad Q,
// naming both of B(k, 2Q), B(k, 2Q + 1) that exist.  Every (quad, k) pair is
// emitted by one thread, so a per-quad cursor in LDS needs no atomics, and
// the barrier after each k keeps every list in ascending k.  Quads are ranked
// within the pair by an LDS bitmap of their column pairs; pairs with more
// quads than kQuadWindow are done in windows.
constexpr int kQuadWindow = 4096;

__device__ inline int64_t qwg_exscan(int64_t v, int64_t *scratch, int64_t *total) {
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    constexpr int nw = kQuadThreads / kWave;
    int64_t x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) scratch[wid] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wid) before += scratch[w];
        all += scratch[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Bitmap of the column pairs Q holding C blocks of rows i0 (and i1) and the
// exclusive popcount prefix per word; returns the number of quads.
__device__ inline int64_t quad_rank_map(const QuadSymArgs &q, int32_t i0, bool two, int nwq,
                                        uint32_t *bits, int32_t *wpre, int64_t *scratch) {
    for (int w = threadIdx.x; w < nwq; w += kQuadThreads) bits[w] = 0u;
    __syncthreads();
    for (int r = 0; r < (two ? 2 : 1); ++r)
        for (int64_t t = q.c_row_ptr[i0 + r] + threadIdx.x; t < q.c_row_ptr[i0 + r + 1];
             t += kQuadThreads) {
            const int32_t Q = q.c_col_idx[t] >> 1;
            atomicOr(&bits[Q >> 5], 1u << (Q & 31));
        }
    __syncthreads();
    const int per = (nwq + kQuadThreads - 1) / kQuadThreads;
    const int w0 = threadIdx.x * per;
    int64_t local = 0;
    for (int w = w0; w < w0 + per && w < nwq; ++w) local += __popc(bits[w]);
    int64_t total;
    int64_t run = qwg_exscan(local, scratch, &total);
    for (int w = w0; w < w0 + per && w < nwq; ++w) {
        wpre[w] = static_cast<int32_t>(run);
        run += __popc(bits[w]);
    }
    __syncthreads();
    return total;
}

// Quads per row pair (one workgroup per pair).
__global__ void __launch_bounds__(kQuadThreads)
k_quad_pairs(QuadSymArgs q, int64_t *cnt) {
    extern __shared__ uint32_t smem[];
    __shared__ int64_t scratch[kQuadThreads / kWave];
    const int nwq = (((q.nbcols + 1) >> 1) + 31) >> 5;
    const int32_t R = blockIdx.x;
    const int32_t i0 = q.r0 + 2 * R;
    const int64_t nq = quad_rank_map(q, i0, i0 + 1 < q.r1, nwq, smem,
                                     reinterpret_cast<int32_t *>(smem + nwq), scratch);
    if (threadIdx.x == 0) cnt[R] = nq;
}

// FILL = false: the quads' C blocks (q_cblk) and entry counts (e_off);
// FILL = true: the entries.
template <bool FILL>
__global__ void __launch_bounds__(kQuadThreads)
k_quad_stack(QuadSymArgs q) {
    extern __shared__ uint32_t smem[];
    __shared__ int64_t scratch[kQuadThreads / kWave];
    __shared__ int64_t s_pa, s_pb;
    __shared__ int32_t s_k, s_a0, s_a1;
    const int nwq = (((q.nbcols + 1) >> 1) + 31) >> 5;   // words of the column-pair bitmap
    uint32_t *bits = smem;
    int32_t *wpre = reinterpret_cast<int32_t *>(smem + nwq);
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + 2 * nwq);
    const int32_t R = blockIdx.x;
    const int32_t i0 = q.r0 + 2 * R, i1 = i0 + 1;
    const bool two = i1 < q.r1;
    quad_rank_map(q, i0, two, nwq, bits, wpre, scratch);

    const int64_t qbase = q.q_off[R], nq = q.q_off[R + 1] - qbase;
    if (!FILL) {
        // C blocks of every quad: (r, c) at 4 quad + 2 r + c, -1 where absent
        for (int64_t t = threadIdx.x; t < 4 * nq; t += kQuadThreads) q.q_cblk[4 * qbase + t] = -1;
        __syncthreads();
        for (int r = 0; r < (two ? 2 : 1); ++r)
            for (int64_t t = q.c_row_ptr[i0 + r] + threadIdx.x; t < q.c_row_ptr[i0 + r + 1];
                 t += kQuadThreads) {
                const int32_t j = q.c_col_idx[t];
                const int64_t rank = bit_rank_q(bits, wpre, j >> 1);
                q.q_cblk[4 * (qbase + rank) + 2 * r + (j & 1)] = t;
                q.q_col[qbase + rank] = j >> 1;    // same value from every block of the quad
            }
    }
    const int64_t ea = q.a_row_ptr[i0 + 1], eb = two ? q.a_row_ptr[i1 + 1] : 0;
    for (int64_t w0 = 0; w0 < nq; w0 += kQuadWindow) {
        const int wn = static_cast<int>(nq - w0 < kQuadWindow ? nq - w0 : kQuadWindow);
        for (int t = threadIdx.x; t < wn; t += kQuadThreads) cnt[t] = 0;
        if (threadIdx.x == 0) {
            s_pa = q.a_row_ptr[i0];
            s_pb = two ? q.a_row_ptr[i1] : 0;
        }
        __syncthreads();
        for (;;) {
            if (threadIdx.x == 0) {
                const int32_t ka = s_pa < ea ? q.a_col_idx[s_pa] : INT_MAX;
                const int32_t kb = s_pb < eb ? q.a_col_idx[s_pb] : INT_MAX;
                const int32_t k = ka < kb ? ka : kb;
                s_k = k;
                s_a0 = (k != INT_MAX && ka == k) ? static_cast<int32_t>(s_pa++) : -1;
                s_a1 = (k != INT_MAX && kb == k) ? static_cast<int32_t>(s_pb++) : -1;
            }
            __syncthreads();
            const int32_t k = s_k;
            if (k == INT_MAX) break;
            const int32_t a0 = s_a0, a1 = s_a1;
            const int64_t tb0 = q.b_row_ptr[k], tb1 = q.b_row_ptr[k + 1];
            for (int64_t tb = tb0 + threadIdx.x; tb < tb1; tb += kQuadThreads) {
                const int32_t j = q.b_col_idx[tb];
                if ((j & 1) && tb > tb0 && q.b_col_idx[tb - 1] == j - 1) continue;  // partner emits
                const int32_t Q = j >> 1;
                const int64_t r = bit_rank_q(bits, wpre, Q) - w0;
                if (r < 0 || r >= wn) continue;
                if (FILL) {
                    int32_t b0 = -1, b1 = -1;
                    if (j & 1) {
                        b1 = static_cast<int32_t>(tb);
                    } else {
                        b0 = static_cast<int32_t>(tb);
                        if (tb + 1 < tb1 && q.b_col_idx[tb + 1] == j + 1) b1 = static_cast<int32_t>(tb + 1);
                    }
                    const int64_t slot = q.e_off[qbase + w0 + r] + cnt[r];
                    q.ent[slot] = make_int4(a0, a1, b0, b1);
                }
                cnt[r] += 1;
            }
            __syncthreads();
        }
        if (!FILL)
            for (int t = threadIdx.x; t < wn; t += kQuadThreads) q.e_off[qbase + w0 + t] = cnt[t];
        __syncthreads();
    }
}

int quad_pairs(const QuadSymArgs &q, int64_t *cnt, hipStream_t s) {
    const int64_t npairs = (static_cast<int64_t>(q.r1 - q.r0) + 1) / 2;
    if (npairs <= 0) return BSM_OK;
    const int nwq = (((q.nbcols + 1) >> 1) + 31) >> 5;
    k_quad_pairs<<<static_cast<unsigned>(npairs), kQuadThreads, sizeof(uint32_t) * 2 * nwq, s>>>(q, cnt);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int quad_stack(const QuadSymArgs &q, bool fill, hipStream_t s) {
    const int64_t npairs = (static_cast<int64_t>(q.r1 - q.r0) + 1) / 2;
    if (npairs <= 0) return BSM_OK;
    const int nwq = (((q.nbcols + 1) >> 1) + 31) >> 5;
    const size_t lds = sizeof(uint32_t) * 2 * nwq + sizeof(int32_t) * kQuadWindow;
    if (fill) k_quad_stack<true><<<static_cast<unsigned>(npairs), kQuadThreads, lds, s>>>(q);
    else k_quad_stack<false><<<static_cast<unsigned>(npairs), kQuadThreads, lds, s>>>(q);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
