// Groups of C blocks with merged product lists (symbolic part of the group
// block-product kernel in smm_quad.hip).  Built straight from the patterns
// of A, B and C, without per-C-block stacks.
//
// A group is the GR x GC set C(GR R + r, GC Q + c), r < GR, c < GC, of the C
// blocks of a chunk (at least one of them present); 2 x 2 groups are the
// quads.  Its entry list is the union of the k's of its C blocks' products,
// ascending; entry k names A(GR R + r, k) for each row r and B(k, GC Q + c)
// for each column c that a product of the group uses, -1 otherwise.  Product
// (r, c) of an entry exists exactly when both A(GR R + r, k) and
// B(k, GC Q + c) are named, so the per-C-block sums are those of the plain
// stacks, in the same (ascending k) order, while every operand block is
// loaded once for up to GC (A) or GR (B) products.  An entry is the GR A
// indices followed by the GC B indices, padded to whole int4.
//
// Mixed block sizes (MAP): the groups are 2 x 2 over paired rows and paired
// columns instead of consecutive ones.  Row group g holds rows rg[2g],
// rg[2g + 1] (the second -1 for a single row), column group Q the columns
// cmap[2Q], cmap[2Q + 1]; the pairs join blocks of equal size (built on the
// host, mixed_pairs below), so every C block of a group has the
// same shape and only k varies between entries.  Entry rules are the same:
// the column of group Q met first in B's row k emits the entry, finding its
// partner column by binary search.
#include <algorithm>
#include <climits>

#include "symbolic.h"

namespace bsm {

constexpr int kQuadThreads = 256;

// Rank of column group Q among the marked bits.
__device__ inline int32_t bit_rank_q(const uint32_t *bits, const int32_t *wpre, int32_t Q) {
    const uint32_t w = bits[Q >> 5];
    const uint32_t below = (Q & 31) ? (w & ((1u << (Q & 31)) - 1u)) : 0u;
    return wpre[Q >> 5] + __popc(below);
}

// ---------------------------------------------------------------------------
// Entry lists straight from the patterns of A and B: one workgroup per row
// group (and k segment) walks k over the merged column lists of A's rows
// GR R .. GR R + GR - 1 (ascending); for each k its threads scan B's row k,
// and the thread holding the first column of group Q present in that row
// emits the entry of group Q, naming every B(k, GC Q + c) that exists.  Every (group, k) pair is
// emitted by one thread, so a per-group cursor in LDS needs no atomics, and
// the barrier after each k keeps every list in ascending k.  Groups are
// ranked within the row group by an LDS bitmap of their column groups; row
// groups with more groups than kQuadWindow are done in windows.
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

__host__ __device__ inline int quad_words(int32_t nbcols, int g) {
    return ((nbcols + g - 1) / g + 31) >> 5;
}
// Words of the column-group bitmap.
__host__ __device__ inline int quad_nwq(const QuadSymArgs &q) {
    return q.map ? (q.ncg + 31) >> 5 : quad_words(q.nbcols, q.gc);
}

// Column group and slot of column j.
template <int GC, bool MAP>
__device__ inline int32_t col_group(const QuadSymArgs &q, int32_t j) {
    return MAP ? q.cgrp[j] : j / GC;
}
template <int GC, bool MAP>
__device__ inline int col_slot(const QuadSymArgs &q, int32_t j) {
    return MAP ? q.cslot[j] : j % GC;
}

// Block row r of row group R of the chunk (-1: none).
template <int GR, bool MAP>
__device__ inline int32_t group_row(const QuadSymArgs &q, int32_t R, int r) {
    if (MAP) return q.rg[GR * (q.g0 + R) + r];
    const int32_t i = q.r0 + GR * R + r;
    return i < q.r1 ? i : -1;
}

// Bitmap of the column groups Q holding C blocks of the rows rows[0..GR)
// (-1: none) and the exclusive popcount prefix per word; returns the number
// of groups.
template <int GR, int GC, bool MAP>
__device__ inline int64_t quad_rank_map(const QuadSymArgs &q, const int32_t (&rows)[GR], int nwq,
                                        uint32_t *bits, int32_t *wpre, int64_t *scratch) {
    for (int w = threadIdx.x; w < nwq; w += kQuadThreads) bits[w] = 0u;
    __syncthreads();
    for (int r = 0; r < GR; ++r) {
        if (rows[r] < 0) continue;
        for (int64_t t = q.c_row_ptr[rows[r]] + threadIdx.x; t < q.c_row_ptr[rows[r] + 1];
             t += kQuadThreads) {
            const int32_t Q = col_group<GC, MAP>(q, q.c_col_idx[t]);
            atomicOr(&bits[Q >> 5], 1u << (Q & 31));
        }
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

// Groups per row group (one workgroup per row group).
template <int GR, int GC, bool MAP>
__global__ void __launch_bounds__(kQuadThreads)
k_quad_pairs(QuadSymArgs q, int64_t *cnt) {
    extern __shared__ uint32_t smem[];
    __shared__ int64_t scratch[kQuadThreads / kWave];
    const int nwq = quad_nwq(q);
    const int32_t R = blockIdx.x;
    int32_t rows[GR];
#pragma unroll
    for (int r = 0; r < GR; ++r) rows[r] = group_row<GR, MAP>(q, R, r);
    const int64_t nq = quad_rank_map<GR, GC, MAP>(q, rows, nwq, smem,
                                                  reinterpret_cast<int32_t *>(smem + nwq), scratch);
    if (threadIdx.x == 0) cnt[R] = nq;
}

// FILL = false: the groups' C blocks (q_cblk) and entry counts (e_off);
// FILL = true: the entries.
template <bool FILL, int GR, int GC, bool MAP>
__global__ void __launch_bounds__(kQuadThreads)
k_quad_stack(QuadSymArgs q) {
    constexpr int GG = GR * GC;
    constexpr int NE = (GR + GC + 3) / 4;          // int4 per entry
    extern __shared__ uint32_t smem[];
    __shared__ int64_t scratch[kQuadThreads / kWave];
    __shared__ int64_t s_tb0, s_tb1;
    __shared__ unsigned long long s_kept;      // fill pass with screening: kept products
    __shared__ int32_t s_k, s_a[GR], s_skip[GR];
    const int nwq = quad_nwq(q);               // words of the column-group bitmap
    uint32_t *bits = smem;
    int32_t *wpre = reinterpret_cast<int32_t *>(smem + nwq);
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + 2 * nwq);
    // fill pass: the window's entry offsets relative to its first group's
    int32_t *eoff = cnt + kQuadWindow;
    __shared__ int64_t s_ebase;
    const int32_t R = blockIdx.x / q.nseg, sg = blockIdx.x % q.nseg;
    int32_t rows[GR];
#pragma unroll
    for (int r = 0; r < GR; ++r) rows[r] = group_row<GR, MAP>(q, R, r);
    // this workgroup's k range
    const int32_t k_lo = sg * q.kseg;
    const int32_t k_hi = (sg == q.nseg - 1) ? INT_MAX : k_lo + q.kseg;
    quad_rank_map<GR, GC, MAP>(q, rows, nwq, bits, wpre, scratch);

    const int64_t qbase = q.q_off[R], nq = q.q_off[R + 1] - qbase;
    if (threadIdx.x == 0) s_kept = 0;
    if (!FILL && sg == 0) {
        // C blocks of every group: (r, c) at GR GC group + GC r + c, -1 where absent
        for (int64_t t = threadIdx.x; t < GG * nq; t += kQuadThreads) q.q_cblk[GG * qbase + t] = -1;
        __syncthreads();
        for (int r = 0; r < GR; ++r) {
            if (rows[r] < 0) continue;
            for (int64_t t = q.c_row_ptr[rows[r]] + threadIdx.x; t < q.c_row_ptr[rows[r] + 1];
                 t += kQuadThreads) {
                const int32_t j = q.c_col_idx[t];
                const int32_t Q = col_group<GC, MAP>(q, j);
                const int64_t rank = bit_rank_q(bits, wpre, Q);
                if (rank >= nq) continue;          // only when q_off was emptied after an overflow
                q.q_cblk[GG * (qbase + rank) + GC * r + col_slot<GC, MAP>(q, j)] = t;
                q.q_col[qbase + rank] = Q;         // same value from every block of the group
            }
        }
    }
    for (int64_t w0 = 0; w0 < nq; w0 += kQuadWindow) {
        const int wn = static_cast<int>(nq - w0 < kQuadWindow ? nq - w0 : kQuadWindow);
        for (int t = threadIdx.x; t < wn; t += kQuadThreads) cnt[t] = 0;
        if (threadIdx.x < GR) s_skip[threadIdx.x] = 0;
        if (FILL) {
            // offsets of this segment's entries for the window's groups (a row
            // group holds fewer than 2^31 entries, so int32 relative offsets)
            if (threadIdx.x == 0) s_ebase = q.e_off[(qbase + w0) * q.nseg + sg];
            __syncthreads();
            for (int t = threadIdx.x; t < wn; t += kQuadThreads)
                eoff[t] = static_cast<int32_t>(q.e_off[(qbase + w0 + t) * q.nseg + sg] - s_ebase);
        }
        __syncthreads();
        // first entry of each A row at or after k_lo: the count of smaller k's
        if (k_lo > 0)
            for (int r = 0; r < GR; ++r) {
                if (rows[r] < 0) continue;
                int32_t c = 0;
                for (int64_t t = q.a_row_ptr[rows[r]] + threadIdx.x; t < q.a_row_ptr[rows[r] + 1];
                     t += kQuadThreads)
                    c += q.a_col_idx[t] < k_lo ? 1 : 0;
                if (c) atomicAdd(&s_skip[r], c);
            }
        __syncthreads();
        // Thread 0 walks the merged A rows one k ahead of the workgroup: the
        // head k of every row, the next k with its A blocks and B row range
        // are in its registers, and the loads behind them are issued one
        // iteration before they are needed.
        int64_t pos[GR], end[GR];
        int32_t head[GR], na[GR];
        int32_t nk = INT_MAX;
        int64_t ntb0 = 0, ntb1 = 0;
        auto advance = [&]() {        // thread 0: the next k from the heads
            nk = INT_MAX;
            for (int r = 0; r < GR; ++r) nk = head[r] < nk ? head[r] : nk;
            for (int r = 0; r < GR; ++r) {
                na[r] = -1;
                if (nk != INT_MAX && head[r] == nk) {
                    na[r] = static_cast<int32_t>(pos[r]++);
                    const int32_t h = pos[r] < end[r] ? q.a_col_idx[pos[r]] : INT_MAX;
                    head[r] = h >= k_hi ? INT_MAX : h;
                }
            }
            if (nk != INT_MAX) {
                ntb0 = q.b_row_ptr[nk];
                ntb1 = q.b_row_ptr[nk + 1];
            }
        };
        if (threadIdx.x == 0) {
            for (int r = 0; r < GR; ++r) {
                pos[r] = rows[r] >= 0 ? q.a_row_ptr[rows[r]] + s_skip[r] : 0;
                end[r] = rows[r] >= 0 ? q.a_row_ptr[rows[r] + 1] : 0;
                const int32_t h = pos[r] < end[r] ? q.a_col_idx[pos[r]] : INT_MAX;
                head[r] = h >= k_hi ? INT_MAX : h;
            }
            advance();
        }
        for (;;) {
            if (threadIdx.x == 0) {
                s_k = nk;
                s_tb0 = ntb0;
                s_tb1 = ntb1;
                for (int r = 0; r < GR; ++r) s_a[r] = na[r];
                if (nk != INT_MAX) advance();
            }
            __syncthreads();
            const int32_t k = s_k;
            if (k == INT_MAX) break;
            const int64_t tb0 = s_tb0, tb1 = s_tb1;
            for (int64_t tb = tb0 + threadIdx.x; tb < tb1; tb += kQuadThreads) {
                const int32_t j = q.b_col_idx[tb];
                const int32_t Q = col_group<GC, MAP>(q, j);
                int64_t partner = -1;          // MAP: B(k, other column of Q), -1 if absent
                if (MAP) {
                    const int sl = col_slot<GC, MAP>(q, j);
                    const int32_t jp = q.cmap[2 * Q + 1 - sl];
                    if (jp >= 0) {
                        int64_t lo = tb0, hi = tb1 - 1;
                        while (lo <= hi) {
                            const int64_t mid = (lo + hi) >> 1;
                            const int32_t cm = q.b_col_idx[mid];
                            if (cm == jp) { partner = mid; break; }
                            if (cm < jp) lo = mid + 1; else hi = mid - 1;
                        }
                    }
                    if (sl == 1 && partner >= 0) continue;            // slot 0 emits
                } else if (tb > tb0 && q.b_col_idx[tb - 1] / GC == Q) {
                    continue;                                         // an earlier column emits
                }
                const int64_t r = bit_rank_q(bits, wpre, Q) - w0;
                if (r < 0 || r >= wn) continue;
                int32_t e[4 * NE];
                unsigned mask = 0;
                if (FILL || q.tau2 > 0.0) {
                    for (int z = 0; z < 4 * NE; ++z) e[z] = -1;
                    for (int r2 = 0; r2 < GR; ++r2) e[r2] = s_a[r2];
                    if (MAP) {
                        const int sl = col_slot<GC, MAP>(q, j);
                        e[GR + sl] = static_cast<int32_t>(tb);
                        if (partner >= 0) e[GR + 1 - sl] = static_cast<int32_t>(partner);
                    } else {
                        for (int64_t t = tb; t < tb1 && t < tb + GC; ++t) {
                            const int32_t jj = q.b_col_idx[t];
                            if (jj / GC != Q) break;
                            e[GR + jj % GC] = static_cast<int32_t>(t);
                        }
                    }
                }
                if (q.tau2 > 0.0) {
                    // screening: keep product (r2, c) only if its norm product
                    // reaches tau^2; operands no kept product uses are dropped
                    for (int r2 = 0; r2 < GR; ++r2)
                        for (int c = 0; c < GC; ++c)
                            if (e[r2] >= 0 && e[GR + c] >= 0 &&
                                q.a_sq[e[r2]] * q.b_sq[e[GR + c]] >= q.tau2)
                                mask |= 1u << (GC * r2 + c);
                    if (mask == 0) continue;
                    for (int r2 = 0; r2 < GR; ++r2)
                        if (((mask >> (GC * r2)) & ((1u << GC) - 1u)) == 0) e[r2] = -1;
                    for (int c = 0; c < GC; ++c) {
                        unsigned colbits = 0;
                        for (int r2 = 0; r2 < GR; ++r2) colbits |= 1u << (GC * r2 + c);
                        if ((mask & colbits) == 0) e[GR + c] = -1;
                    }
                }
                if (FILL) {
                    const int64_t slot = s_ebase + eoff[r] + cnt[r];
                    for (int h = 0; h < NE; ++h)
                        q.ent[NE * slot + h] = make_int4(e[4 * h], e[4 * h + 1], e[4 * h + 2], e[4 * h + 3]);
                    if (q.tau2 > 0.0) {
                        q.pm[slot] = static_cast<int32_t>(mask);
                        atomicAdd(&s_kept, static_cast<unsigned long long>(__popc(mask)));
                    }
                }
                cnt[r] += 1;
            }
            __syncthreads();
        }
        if (!FILL)
            for (int t = threadIdx.x; t < wn; t += kQuadThreads)
                q.e_off[(qbase + w0 + t) * q.nseg + sg] = cnt[t];
        __syncthreads();
    }
    if (FILL && q.tau2 > 0.0 && threadIdx.x == 0 && s_kept) atomicAdd(q.kept, s_kept);
}

#define BSM_QUAD_SHAPES(X) X(2, 2) X(4, 4) X(4, 2)

static int64_t quad_groups(const QuadSymArgs &q) {
    return q.map ? q.ngroups : (static_cast<int64_t>(q.r1 - q.r0) + q.gr - 1) / q.gr;
}

int quad_pairs(const QuadSymArgs &q, int64_t *cnt, hipStream_t s) {
    const int64_t ngroups = quad_groups(q);
    if (ngroups <= 0) return BSM_OK;
    const size_t lds = sizeof(uint32_t) * 2 * quad_nwq(q);
    const unsigned g = static_cast<unsigned>(ngroups);
    if (q.map) {
        if (q.gr != 2 || q.gc != 2) { set_error("internal: mixed groups are 2 x 2"); return BSM_EINVAL; }
        k_quad_pairs<2, 2, true><<<g, kQuadThreads, lds, s>>>(q, cnt);
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
#define BSM_QP(R_, C_) \
    if (q.gr == R_ && q.gc == C_) { k_quad_pairs<R_, C_, false><<<g, kQuadThreads, lds, s>>>(q, cnt); BSM_HIP(hipGetLastError()); return BSM_OK; }
    BSM_QUAD_SHAPES(BSM_QP)
#undef BSM_QP
    set_error("internal: no %d x %d group builder", q.gr, q.gc);
    return BSM_EINVAL;
}

int quad_stack(const QuadSymArgs &q, bool fill, hipStream_t s) {
    const int64_t ngroups = quad_groups(q);
    if (ngroups <= 0) return BSM_OK;
    if (q.nseg < 1 || q.kseg < 1) { set_error("internal: quad k segments"); return BSM_EINVAL; }
    const size_t lds = sizeof(uint32_t) * 2 * quad_nwq(q) +
                       sizeof(int32_t) * kQuadWindow * (fill ? 2 : 1);
    const int64_t nblk = ngroups * q.nseg;
    if (nblk > (1ll << 31) - 1) { set_error("too many row groups in one chunk"); return BSM_EINVAL; }
    const unsigned g = static_cast<unsigned>(nblk);
    if (q.map) {
        if (q.gr != 2 || q.gc != 2) { set_error("internal: mixed groups are 2 x 2"); return BSM_EINVAL; }
        if (fill) k_quad_stack<true, 2, 2, true><<<g, kQuadThreads, lds, s>>>(q);
        else k_quad_stack<false, 2, 2, true><<<g, kQuadThreads, lds, s>>>(q);
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
#define BSM_QS(R_, C_)                                                                     \
    if (q.gr == R_ && q.gc == C_) {                                                        \
        if (fill) k_quad_stack<true, R_, C_, false><<<g, kQuadThreads, lds, s>>>(q);       \
        else k_quad_stack<false, R_, C_, false><<<g, kQuadThreads, lds, s>>>(q);           \
        BSM_HIP(hipGetLastError());                                                        \
        return BSM_OK;                                                                     \
    }
    BSM_QUAD_SHAPES(BSM_QS)
#undef BSM_QS
    set_error("internal: no %d x %d group builder", q.gr, q.gc);
    return BSM_EINVAL;
}

__global__ void k_seg_starts(const int64_t *seg_off, int32_t nseg, int64_t n, int64_t *starts) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g <= n) starts[g] = seg_off[g * nseg];
}

int quad_seg_starts(const int64_t *seg_off, int32_t nseg, int64_t n_groups, int64_t *starts,
                    hipStream_t s) {
    k_seg_starts<<<grid_for(n_groups + 1, 256), 256, 0, s>>>(seg_off, nseg, n_groups, starts);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// Pairs of equal-size block rows (within bands of kPairBand rows, so that
// chunk cuts at band edges never split a pair) and of equal-size block
// columns (over all columns), for the mixed-size groups: rows of each size
// in ascending order are paired in turn, the last one alone when their count
// is odd; groups are listed by their first row (column).  band_g0[b] is the
// first row group of band b.
void mixed_pairs(const std::vector<int32_t> &rbs, const std::vector<int32_t> &cbs, MixedPairs *mp) {
    const int32_t nbr = static_cast<int32_t>(rbs.size()), nbc = static_cast<int32_t>(cbs.size());
    mp->rg.clear();
    mp->band_g0.clear();
    for (int32_t b0 = 0; b0 < nbr; b0 += kPairBand) {
        mp->band_g0.push_back(static_cast<int32_t>(mp->rg.size() / 2));
        const int32_t b1 = std::min(nbr, b0 + kPairBand);
        std::vector<int32_t> open(kMaxBlock + 1, -1);     // unpaired row of each size
        std::vector<std::pair<int32_t, int32_t>> groups;
        for (int32_t i = b0; i < b1; ++i) {
            int32_t &o = open[rbs[i]];
            if (o < 0) { o = i; continue; }
            groups.push_back({o, i});
            o = -1;
        }
        for (int32_t v : open)
            if (v >= 0) groups.push_back({v, -1});
        std::sort(groups.begin(), groups.end());
        for (auto &g : groups) { mp->rg.push_back(g.first); mp->rg.push_back(g.second); }
    }
    mp->band_g0.push_back(static_cast<int32_t>(mp->rg.size() / 2));
    std::vector<int32_t> open(kMaxBlock + 1, -1);
    std::vector<std::pair<int32_t, int32_t>> groups;
    for (int32_t j = 0; j < nbc; ++j) {
        int32_t &o = open[cbs[j]];
        if (o < 0) { o = j; continue; }
        groups.push_back({o, j});
        o = -1;
    }
    for (int32_t v : open)
        if (v >= 0) groups.push_back({v, -1});
    std::sort(groups.begin(), groups.end());
    mp->cgrp.assign(nbc, -1);
    mp->cslot.assign(nbc, 0);
    mp->cmap.clear();
    for (size_t q = 0; q < groups.size(); ++q) {
        mp->cmap.push_back(groups[q].first);
        mp->cmap.push_back(groups[q].second);
        mp->cgrp[groups[q].first] = static_cast<int32_t>(q);
        mp->cslot[groups[q].first] = 0;
        if (groups[q].second >= 0) {
            mp->cgrp[groups[q].second] = static_cast<int32_t>(q);
            mp->cslot[groups[q].second] = 1;
        }
    }
}

}  // namespace bsm
