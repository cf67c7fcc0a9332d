// Numeric phase of the block-sparse multiply: execute the product stacks.
//
// The paper's GPU driver runs batches of small dense block products
// C_blk += A_blk * B_blk with coalesced loads ("Batched execution"
// subsection).  Here the batches are C-stationary: one wavefront owns one C
// block, walks its segment of products (ascending k), keeps the sum in
// registers and writes alpha*sum + beta*C_in once, together with the block's
// squared Frobenius norm and max |x| for the filter.  No atomics, fixed
// summation order.
//
// FP64 path: the block products run on the CDNA matrix cores, mainly with
// V_MFMA_F64_4X4X4_4B_F64.  Operand blocks are staged through LDS with
// contiguous (coalesced) global loads, then read in MFMA operand layout.
// This file holds the compile-time-shape kernels (uniform sizes, per-(m, n)
// class), the run-time-shape code path used by the fused persistent launch,
// and the launch dispatch; smm_rt.hip holds the tunable run-time-shape
// kernels and smm_lowp.hip the reduced-precision ones.
#include "smm.h"

namespace bsm {

typedef double d4 __attribute__((ext_vector_type(4)));

// Work item of workgroup g: consecutive items go to the same XCD (the
// hardware hands workgroup g to XCD g % 8), so C blocks of one block row --
// which read the same A blocks -- share that XCD's L2.
__device__ inline int64_t xcd_item(int64_t n_items) {
    const int64_t per = (n_items + kXcds - 1) / kXcds;
    return static_cast<int64_t>(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

// A value that is the same in every lane (read from LDS at a uniform
// address), made wave-uniform for the compiler.
__device__ inline int64_t uniform64(int64_t v) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v)));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32)));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ inline double wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// ---------------------------------------------------------------------------
// Run-time-shape C-block code path on V_MFMA_F64_4X4X4_4B_F64 (four
// independent 4x4x4 products per instruction), used by the fused persistent
// launch.  On gfx950 this instruction sustains ~95% of the FP64 peak, and its
// 4-wide tiles pad a 23 x 23 block only to 24 x 24.
//
// Lane layout (measured on gfx950): lane = 16*x + 4*b + y, b = block 0..3;
// A_b(i,k): x = k, y = i;  B_b(k,j): x = k, y = j;  D_b(i,j): x = i, y = j.
//
// The C block (m, n <= 32) is cut into 4-row / 4-column tiles; instruction
// block b = 2*bh + bw owns the tiles of row half bh and column half bw, so
// each lane holds RT x CT accumulators (one element per tile).  Per k-step a
// lane reads RT A values and CT B values from LDS and issues RT*CT MFMAs.
// The next product's two operand blocks are prefetched into registers with
// contiguous loads while the current one is multiplied.
template <int RT, int CT>
__device__ inline void m4_cblock(const SmmArgs &a, int64_t c, double *sm) {
    constexpr int kMaxM = 8 * RT, kMaxN = 8 * CT, kMaxK = kMaxBlock;
    constexpr int NA = (kMaxM * kMaxK + kWave - 1) / kWave;   // A doubles per lane
    constexpr int NB = (kMaxK * kMaxN + kWave - 1) / kWave;   // B doubles per lane
    const int lane = threadIdx.x;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3;
    const int bh = blk >> 1, bw = blk & 1;
    const int m = a.c_rbs[a.c_row[c]], n = a.c_cbs[a.c_col[c]];
    const int hr = (((m + 3) >> 2) + 1) >> 1;      // row tiles per half
    const int hc = (((n + 3) >> 2) + 1) >> 1;      // column tiles per half
    double *sA = sm;
    double *sB = sm + a.max_m * a.max_k;

    double acc[RT][CT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u) acc[t][u] = 0.0;

    const int64_t p0 = a.seg[c - a.c0], p_end = a.seg[c - a.c0 + 1];
    double ra[NA], rb[NB];
    int k_next = 0;
    auto prefetch = [&](int64_t p) {
        const int32_t ta = a.stk_a[p], tb = a.stk_b[p];
        k_next = a.k_size[a.a_col_idx[ta]];
        const double *ga = a.a_vals + a.a_blk_off[ta];
        const double *gb = a.b_vals + a.b_blk_off[tb];
        const int na = m * k_next, nb = k_next * n;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = lane + q * kWave;
            ra[q] = (e < na) ? ga[e] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = lane + q * kWave;
            rb[q] = (e < nb) ? gb[e] : 0.0;
        }
    };
    if (p0 < p_end) prefetch(p0);
    for (int64_t p = p0; p < p_end; ++p) {
        const int k = k_next;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = lane + q * kWave;
            if (e < m * k) sA[e] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = lane + q * kWave;
            if (e < k * n) sB[e] = rb[q];
        }
        __syncthreads();
        if (p + 1 < p_end) prefetch(p + 1);
        for (int ks = 0; ks < k; ks += 4) {
            const int kk = ks + x;
            double av[RT], bv[CT];
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int r = 4 * (bh * hr + t) + y;
                av[t] = (t < hr && r < m && kk < k) ? sA[r * k + kk] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CT; ++u) {
                const int cc = 4 * (bw * hc + u) + y;
                bv[u] = (u < hc && cc < n && kk < k) ? sB[kk * n + cc] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int u = 0; u < CT; ++u)
                    if (t < hr && u < hc)
                        acc[t][u] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[t], bv[u], acc[t][u],
                                                                       0, 0, 0);
        }
        __syncthreads();
    }

    // epilogue: alpha*acc + beta*C_in, store, block norms
    const int64_t co = a.c_blk_off[c];
    const double *cin = nullptr;
    if (a.cin_map) {
        const int64_t t = a.cin_map[c];
        if (t >= 0) cin = a.cin_vals + a.cin_blk_off[t];
    }
    double sq = 0.0, mx = 0.0;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u) {
            const int row = 4 * (bh * hr + t) + x, col = 4 * (bw * hc + u) + y;
            if (t < hr && u < hc && row < m && col < n) {
                double v = a.alpha * acc[t][u];
                if (cin) v += a.beta * cin[row * n + col];
                a.c_vals[co + row * n + col] = v;
                sq += v * v;
                mx = fmax(mx, fabs(v));
            }
        }
    sq = wave_sum(sq);
    mx = wave_max(mx);
    if (lane == 0) {
        a.sq_out[c] = sq;
        a.mx_out[c] = mx;
        if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
    }
    __syncthreads();   // LDS is reused by the next C block of a persistent wave
}

// ---------------------------------------------------------------------------
// FP64 kernel for uniform block sizes known at compile time (M x K times
// K x N).  Same instruction and lane roles as the run-time-shape 4 x 4-tile
// path (m4_cblock), but:
//  * the operand blocks sit in LDS exactly as in HBM (A then B, row-major,
//    followed by a zeroed tail), so staging is a contiguous copy with
//    immediate offsets and needs no per-lane index registers;
//  * the k loop is fully unrolled with immediate LDS offsets;
//  * only the k-padding lanes of the last k-step are masked: padding rows of
//    A and padding columns of B just read neighbouring data, which reaches
//    only accumulator rows/columns that are never stored.
// Odd K and N (5, 13, 23) keep the rows one instruction reads in distinct
// LDS banks.
template <int M, int N, int K>
struct FixedShape {
    static constexpr int MT = (M + 3) / 4, NT = (N + 3) / 4, KS = (K + 3) / 4;
    static constexpr int HR = (MT + 1) / 2, HC = (NT + 1) / 2;
    static constexpr int KLAST = K - 4 * (KS - 1);     // valid x in the last k-step
    static constexpr int TAIL = 4 * K + 8 * N + 8;     // covers padded reads past B
    static constexpr int SIZE = M * K + K * N + TAIL;
    static constexpr int NA = (M * K + kWave - 1) / kWave;
    static constexpr int NB = (K * N + kWave - 1) / kWave;
};

// WPE: the occupancy (waves per SIMD) the register allocation aims for.
template <int M, int N, int K, int WPE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_smm_f64_fixed(SmmArgs a) {
    using S = FixedShape<M, N, K>;
    __shared__ double sm[S::SIZE];
    double *sA = sm;
    double *sB = sm + M * K;
    const int64_t item = xcd_item(a.nC);
    if (item >= a.nC) return;
    const int lane = threadIdx.x;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3;
    const int bh = blk >> 1, bw = blk & 1;
    const int64_t c = a.worklist ? a.worklist[a.c0 + item] : a.c0 + item;

    for (int e = M * K + K * N + lane; e < S::SIZE; e += kWave) sm[e] = 0.0;
    const int ra0 = (4 * bh * S::HR + y) * K + x;      // A(4*(bh*HR+t)+y, 4*ks+x)
    const int rb0 = x * N + 4 * bw * S::HC + y;        // B(4*ks+x, 4*(bw*HC+u)+y)
    const bool klast_ok = x < S::KLAST;

    double acc[S::HR][S::HC];
#pragma unroll
    for (int t = 0; t < S::HR; ++t)
#pragma unroll
        for (int u = 0; u < S::HC; ++u) acc[t][u] = 0.0;

    const int64_t p0 = a.seg[c - a.c0], p_end = a.seg[c - a.c0 + 1];
    double pa[S::NA], pb[S::NB];
    auto prefetch = [&](int64_t p) {
        const double *ga = a.a_vals + a.a_blk_off[a.stk_a[p]];
        const double *gb = a.b_vals + a.b_blk_off[a.stk_b[p]];
#pragma unroll
        for (int q = 0; q < S::NA; ++q)
            if (q < S::NA - 1 || lane + q * kWave < M * K) pa[q] = ga[lane + q * kWave];
#pragma unroll
        for (int q = 0; q < S::NB; ++q)
            if (q < S::NB - 1 || lane + q * kWave < K * N) pb[q] = gb[lane + q * kWave];
    };
    if (p0 < p_end) prefetch(p0);
    for (int64_t p = p0; p < p_end; ++p) {
#pragma unroll
        for (int q = 0; q < S::NA; ++q)
            if (q < S::NA - 1 || lane + q * kWave < M * K) sA[lane + q * kWave] = pa[q];
#pragma unroll
        for (int q = 0; q < S::NB; ++q)
            if (q < S::NB - 1 || lane + q * kWave < K * N) sB[lane + q * kWave] = pb[q];
        __syncthreads();
        if (p + 1 < p_end) prefetch(p + 1);
#pragma unroll
        for (int ks = 0; ks < S::KS; ++ks) {
            double av[S::HR], bv[S::HC];
#pragma unroll
            for (int t = 0; t < S::HR; ++t) av[t] = sA[ra0 + 4 * t * K + 4 * ks];
#pragma unroll
            for (int u = 0; u < S::HC; ++u) bv[u] = sB[rb0 + 4 * u + 4 * ks * N];
            if (ks == S::KS - 1 && S::KLAST < 4) {
#pragma unroll
                for (int t = 0; t < S::HR; ++t) av[t] = klast_ok ? av[t] : 0.0;
#pragma unroll
                for (int u = 0; u < S::HC; ++u) bv[u] = klast_ok ? bv[u] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < S::HR; ++t)
#pragma unroll
                for (int u = 0; u < S::HC; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[t], bv[u], acc[t][u], 0, 0, 0);
        }
        __syncthreads();
    }

    const int64_t co = a.c_blk_off[c];
    const double *cin = nullptr;
    if (a.cin_map) {
        const int64_t t = a.cin_map[c];
        if (t >= 0) cin = a.cin_vals + a.cin_blk_off[t];
    }
    double sq = 0.0, mx = 0.0;
#pragma unroll
    for (int t = 0; t < S::HR; ++t)
#pragma unroll
        for (int u = 0; u < S::HC; ++u) {
            const int row = 4 * (bh * S::HR + t) + x, col = 4 * (bw * S::HC + u) + y;
            if (row < M && col < N) {
                double v = a.alpha * acc[t][u];
                if (cin) v += a.beta * cin[row * N + col];
                a.c_vals[co + row * N + col] = v;
                sq += v * v;
                mx = fmax(mx, fabs(v));
            }
        }
    sq = wave_sum(sq);
    mx = wave_max(mx);
    if (lane == 0) {
        a.sq_out[c] = sq;
        a.mx_out[c] = mx;
        if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
    }
}

// ---------------------------------------------------------------------------
// Per-(m, n)-class FP64 kernel with run-time k: M and N are compile-time, the
// k of each product is read from the stack.  Launched once per class over the
// class's contiguous range of the class-sorted work list.  LDS holds the two
// operand blocks contiguously (as in HBM) plus a zeroed tail; lanes whose k
// index passes the product's k read zero.
constexpr int kClassKmax = 26;   // largest k of the class set {5, 13, 23, 26}


// Staging and multiply of one product with k known at compile time (the
// class set's k in {5, 13, 23, 26}): fully unrolled k-steps, only the last
// one masked.  Layout as in k_smm_f64_class: A (M x K) then B (K x N),
// row-major, then the zeroed tail; padded rows/columns read neighbouring
// data that reaches only accumulator elements that are never stored.
template <int M, int N, int K, int NA, int NB, int TAIL>
__device__ inline void class_stage(double *sm, int lane, const double (&pa)[NA],
                                   const double (&pb)[NB]) {
    double *sA = sm, *sB = sm + M * K;
#pragma unroll
    for (int v = 0; v < NA; ++v)
        if (v * kWave < M * K && lane + v * kWave < M * K) sA[lane + v * kWave] = pa[v];
#pragma unroll
    for (int v = 0; v < NB; ++v)
        if (v * kWave < K * N && lane + v * kWave < K * N) sB[lane + v * kWave] = pb[v];
#pragma unroll
    for (int e = M * K + K * N; e < M * K + K * N + TAIL; e += kWave)
        if (e + lane < M * K + K * N + TAIL) sm[e + lane] = 0.0;
}

template <int M, int N, int K, int HR, int HC>
__device__ inline void class_compute(const double *sm, int bh, int bw, int x, int y,
                                     double (&acc)[HR][HC]) {
    constexpr int KS = (K + 3) / 4, KLAST = K - 4 * (KS - 1);
    const double *sA = sm, *sB = sm + M * K;
    const int ra0 = (4 * bh * HR + y) * K + x, rb0 = x * N + 4 * bw * HC + y;
    const bool ok = x < KLAST;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        double av[HR], bv[HC];
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const double v = sA[ra0 + 4 * t * K + 4 * ks];
            av[t] = (ks == KS - 1 && KLAST < 4 && !ok) ? 0.0 : v;
        }
#pragma unroll
        for (int u = 0; u < HC; ++u) {
            const double v = sB[rb0 + 4 * u + 4 * ks * N];
            bv[u] = (ks == KS - 1 && KLAST < 4 && !ok) ? 0.0 : v;
        }
#pragma unroll
        for (int t = 0; t < HR; ++t)
#pragma unroll
            for (int u = 0; u < HC; ++u)
                acc[t][u] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[t], bv[u], acc[t][u], 0, 0, 0);
    }
}

// LDS of one class C block: the two operand blocks, a zeroed tail and the
// product metadata of the per-class kernel.
template <int N>
constexpr int class_tail() { return 4 * kClassKmax + 8 * N + 8; }
constexpr int kMetaChunk = 64;
struct ClassMeta {
    int64_t off[2][2][kMetaChunk];   // [buffer][A, B][product]
    int32_t k[2][kMetaChunk];
};

// C block c of class (M, N) on one wavefront (the per-class kernel's body).
template <int M, int N>
__device__ inline void class_cblock(const SmmArgs &a, int64_t c, double *sm, ClassMeta &md) {
    constexpr int MT = (M + 3) / 4, NT = (N + 3) / 4;
    constexpr int HR = (MT + 1) / 2, HC = (NT + 1) / 2;
    constexpr int NA = (M * kClassKmax + kWave - 1) / kWave;
    constexpr int NB = (kClassKmax * N + kWave - 1) / kWave;
    constexpr int TAIL = class_tail<N>();
    const int lane = threadIdx.x;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3;
    const int bh = blk >> 1, bw = blk & 1;
    double acc[HR][HC];
#pragma unroll
    for (int t = 0; t < HR; ++t)
#pragma unroll
        for (int u = 0; u < HC; ++u) acc[t][u] = 0.0;
    // Per-product metadata (operand offsets and k) is fetched for 64 products
    // at once, one product per lane, and kept in LDS (double-buffered; the next
    // chunk waits in registers), so the operand loads of product p + 1 never
    // wait on the chain stack -> block index -> offset of the same iteration.
    auto &m_off = md.off;
    auto &m_k = md.k;
    const int64_t p0 = a.seg[c - a.c0], np = a.seg[c - a.c0 + 1] - p0;
    int64_t r_aoff = 0, r_boff = 0;
    int r_k = 0;
    auto meta = [&](int64_t q, int64_t &ao, int64_t &bo, int &kk) {   // q < np
        const int32_t ta = a.stk_a[p0 + q];
        ao = a.a_blk_off[ta];
        bo = a.b_blk_off[a.stk_b[p0 + q]];
        kk = a.k_size[a.a_col_idx[ta]];
    };
    if (lane < np) {
        int64_t ao, bo;
        int kk;
        meta(lane, ao, bo, kk);
        m_off[0][0][lane] = ao;
        m_off[0][1][lane] = bo;
        m_k[0][lane] = kk;
    }
    if (kMetaChunk + lane < np) meta(kMetaChunk + lane, r_aoff, r_boff, r_k);
    __syncthreads();
    double pa[NA], pb[NB];
    int kn = 0;
    auto prefetch = [&](int64_t q) {           // operand blocks of product q (from LDS metadata)
        const int buf = static_cast<int>((q / kMetaChunk) & 1), i = static_cast<int>(q % kMetaChunk);
        kn = __builtin_amdgcn_readfirstlane(m_k[buf][i]);
        const double *gA = a.a_vals + uniform64(m_off[buf][0][i]);
        const double *gB = a.b_vals + uniform64(m_off[buf][1][i]);
#pragma unroll
        for (int v = 0; v < NA; ++v)
            if (lane + v * kWave < M * kn) pa[v] = gA[lane + v * kWave];
#pragma unroll
        for (int v = 0; v < NB; ++v)
            if (lane + v * kWave < kn * N) pb[v] = gB[lane + v * kWave];
    };
    if (np > 0) prefetch(0);
    for (int64_t t = 0; t < np; ++t) {
        const int k = kn;
        double *sA = sm, *sB = sm + M * k;
        switch (k) {
            case 5: class_stage<M, N, 5, NA, NB, TAIL>(sm, lane, pa, pb); break;
            case 13: class_stage<M, N, 13, NA, NB, TAIL>(sm, lane, pa, pb); break;
            case 23: class_stage<M, N, 23, NA, NB, TAIL>(sm, lane, pa, pb); break;
            case 26: class_stage<M, N, 26, NA, NB, TAIL>(sm, lane, pa, pb); break;
            default:
#pragma unroll
                for (int v = 0; v < NA; ++v)
                    if (lane + v * kWave < M * k) sA[lane + v * kWave] = pa[v];
#pragma unroll
                for (int v = 0; v < NB; ++v)
                    if (lane + v * kWave < k * N) sB[lane + v * kWave] = pb[v];
                for (int e = M * k + k * N + lane; e < M * k + k * N + TAIL; e += kWave) sm[e] = 0.0;
        }
        const int64_t t1 = t + 1;
        if ((t1 % kMetaChunk) == 0 && t1 < np) {
            const int buf = static_cast<int>((t1 / kMetaChunk) & 1);
            m_off[buf][0][lane] = r_aoff;
            m_off[buf][1][lane] = r_boff;
            m_k[buf][lane] = r_k;
            if (t1 + kMetaChunk + lane < np) meta(t1 + kMetaChunk + lane, r_aoff, r_boff, r_k);
        }
        __syncthreads();
        if (t1 < np) prefetch(t1);
        switch (k) {
            case 5: class_compute<M, N, 5, HR, HC>(sm, bh, bw, x, y, acc); break;
            case 13: class_compute<M, N, 13, HR, HC>(sm, bh, bw, x, y, acc); break;
            case 23: class_compute<M, N, 23, HR, HC>(sm, bh, bw, x, y, acc); break;
            case 26: class_compute<M, N, 26, HR, HC>(sm, bh, bw, x, y, acc); break;
            default: {
                int ra[HR];
#pragma unroll
                for (int t = 0; t < HR; ++t) ra[t] = (4 * (bh * HR + t) + y) * k + x;
                const int rb = x * N + 4 * bw * HC + y;
#pragma unroll 1
                for (int ks = 0; 4 * ks < k; ++ks) {
                    const bool ok = 4 * ks + x < k;
                    double av[HR], bv[HC];
#pragma unroll
                    for (int t = 0; t < HR; ++t) av[t] = ok ? sA[ra[t] + 4 * ks] : 0.0;
#pragma unroll
                    for (int u = 0; u < HC; ++u) bv[u] = ok ? sB[rb + 4 * u + 4 * ks * N] : 0.0;
#pragma unroll
                    for (int t = 0; t < HR; ++t)
#pragma unroll
                        for (int u = 0; u < HC; ++u)
                            acc[t][u] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[t], bv[u], acc[t][u], 0, 0, 0);
                }
            }
        }
        __syncthreads();                       // this product's reads are done
    }
    const int64_t co = a.c_blk_off[c];
    const double *cin = nullptr;
    if (a.cin_map) {
        const int64_t t = a.cin_map[c];
        if (t >= 0) cin = a.cin_vals + a.cin_blk_off[t];
    }
    double sq = 0.0, mx = 0.0;
#pragma unroll
    for (int t = 0; t < HR; ++t)
#pragma unroll
        for (int u = 0; u < HC; ++u) {
            const int row = 4 * (bh * HR + t) + x, col = 4 * (bw * HC + u) + y;
            if (row < M && col < N) {
                double v = a.alpha * acc[t][u];
                if (cin) v += a.beta * cin[row * N + col];
                a.c_vals[co + row * N + col] = v;
                sq += v * v;
                mx = fmax(mx, fabs(v));
            }
        }
    sq = wave_sum(sq);
    mx = wave_max(mx);
    if (lane == 0) {
        a.sq_out[c] = sq;
        a.mx_out[c] = mx;
        if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
    }
}

template <int M, int N>
__global__ void __launch_bounds__(64)
k_smm_f64_class(SmmArgs a) {
    __shared__ double sm[M * kClassKmax + kClassKmax * N + class_tail<N>()];
    __shared__ ClassMeta md;
    const int64_t item = xcd_item(a.nC);
    if (item >= a.nC) return;
    class_cblock<M, N>(a, a.worklist[a.c0 + item], sm, md);
}

int class_of_size(int b) { return b == 5 ? 0 : b == 13 ? 1 : b == 23 ? 2 : b == 26 ? 3 : -1; }

int launch_class(const SmmArgs &a, int cls, hipStream_t s) {
    if (a.nC <= 0) return BSM_OK;
    const int64_t per = (a.nC + kXcds - 1) / kXcds;
    const unsigned grid = static_cast<unsigned>(per * kXcds);
    switch (cls) {
#define BSM_CL(ID, MM, NN) case ID: BSM_LAUNCH((k_smm_f64_class<MM, NN>), grid, 64, 0, s)(a); break;
        BSM_CL(0, 5, 5) BSM_CL(1, 5, 13) BSM_CL(2, 5, 23) BSM_CL(3, 5, 26)
        BSM_CL(4, 13, 5) BSM_CL(5, 13, 13) BSM_CL(6, 13, 23) BSM_CL(7, 13, 26)
        BSM_CL(8, 23, 5) BSM_CL(9, 23, 13) BSM_CL(10, 23, 23) BSM_CL(11, 23, 26)
        BSM_CL(12, 26, 5) BSM_CL(13, 26, 13) BSM_CL(14, 26, 23) BSM_CL(15, 26, 26)
#undef BSM_CL
        default: set_error("no class kernel %d", cls); return BSM_EINVAL;
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// ---------------------------------------------------------------------------
// Fused persistent FP64 kernel: a fixed grid of single-wave workgroups drains
// the whole work list of a chunk -- every (m, n) class -- through an atomic
// counter, running the run-time-shape 4 x 4-tile code path for each C block.
// The list is sorted by descending cost (largest stacks first), so the tail
// of the launch is short.  Every wave exits when the counter passes the end.
__global__ void __launch_bounds__(64)
k_smm_f64_persistent(SmmArgs a, unsigned long long *counter) {
    extern __shared__ double sm[];
    for (;;) {
        int64_t item = 0;
        if (threadIdx.x == 0) item = static_cast<int64_t>(atomicAdd(counter, 1ull));
        item = __shfl(item, 0, kWave);
        if (item >= a.nC) break;
        m4_cblock<4, 4>(a, a.worklist ? a.worklist[a.c0 + item] : a.c0 + item, sm);
    }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

static int launch_persistent(const SmmArgs &a, hipStream_t s) {
    int dev = 0, cus = 256;
    BSM_HIP(hipGetDevice(&dev));
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t lds = sizeof(double) * (static_cast<size_t>(a.max_m) * a.max_k +
                                         static_cast<size_t>(a.max_k) * a.max_n);
    unsigned long long *counter = a.counter;
    if (!counter) BSM_TRY(dalloc(&counter, 1, s));
    k_zero_u64<<<1, 1, 0, s>>>(counter);
    const int64_t want = static_cast<int64_t>(cus) * 8;    // 2 waves per SIMD (its occupancy)
    const unsigned grid = static_cast<unsigned>(want < a.nC ? want : a.nC);
    BSM_LAUNCH((k_smm_f64_persistent), grid, 64, lds, s)(a, counter);
    const hipError_t e = hipGetLastError();
    if (!a.counter) dfree(counter, s);
    if (e != hipSuccess) { set_error("persistent launch: %s", hipGetErrorString(e)); return BSM_EDEVICE; }
    return BSM_OK;
}

// Uniform (m, n, k) shapes with a compile-time kernel.
bool smm_fixed_available(int m, int n, int k) {
    return (m == n && n == k) && (m == 5 || m == 6 || m == 13 || m == 23 || m == 26 || m == 32);
}

int launch_fixed(const SmmArgs &a, int m, unsigned grid, hipStream_t s) {
    switch (m) {
        case 5: BSM_LAUNCH((k_smm_f64_fixed<5, 5, 5, 8>), grid, 64, 0, s)(a); break;
        case 6: BSM_LAUNCH((k_smm_f64_fixed<6, 6, 6, 8>), grid, 64, 0, s)(a); break;
        case 13: BSM_LAUNCH((k_smm_f64_fixed<13, 13, 13, 8>), grid, 64, 0, s)(a); break;
        case 23: BSM_LAUNCH((k_smm_f64_fixed<23, 23, 23, 4>), grid, 64, 0, s)(a); break;
        case 26: BSM_LAUNCH((k_smm_f64_fixed<26, 26, 26, 3>), grid, 64, 0, s)(a); break;
        case 32: BSM_LAUNCH((k_smm_f64_fixed<32, 32, 32, 2>), grid, 64, 0, s)(a); break;
        default: set_error("no fixed-shape kernel for %d", m); return BSM_EINVAL;
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// Tuned parameters for a launch whose shapes are (max_m, max_n, max_k), or
// the uniform sizes when they are uniform; defaults when the table has none.
static SmmParams tuned_params(const SmmArgs &a) {
    SmmParams p{1, 1, 1, 0};
    if (a.uni_m && a.uni_n && a.uni_k) {
        if (table_lookup(a.uni_m, a.uni_n, a.uni_k, &p) && p.family != 2) return p;
        return SmmParams{1, 1, 1, 0};
    }
    SmmParams q;
    if (table_lookup(a.max_m, a.max_n, 0, &q) && q.family != 2) return q;
    return p;
}

int smm_launch(const SmmArgs &a, int variant, hipStream_t s) {
    if (a.nC <= 0) return BSM_OK;
    const int64_t per = (a.nC + kXcds - 1) / kXcds;
    const int64_t grid = per * kXcds;
    if (grid > (1ll << 31) - 1) {
        set_error("too many C blocks in one launch (%lld)", (long long)a.nC);
        return BSM_EINVAL;
    }
    switch (variant) {
        case kSmmF64M16: return launch_rt(a, SmmParams{0, 1, 0, 0}, s);
        case kSmmF64M4: return launch_rt(a, SmmParams{1, 1, 1, 0}, s);
        case kSmmF64Quad:   // where the quad kernel does not apply (built by multiply)
        case kSmmF64Fixed: {
            // uniform sizes: the tuning table may choose the family; without
            // an entry the compile-time-shape kernel is used where it exists
            const bool uni = a.uni_m && a.uni_n && a.uni_k;
            SmmParams p;
            const bool have = uni && table_lookup(a.uni_m, a.uni_n, a.uni_k, &p);
            if (have && p.family == 2 && class_of_size(a.uni_m) >= 0 && class_of_size(a.uni_n) >= 0 &&
                a.uni_k <= 26 && a.worklist)
                return launch_class(a, 4 * class_of_size(a.uni_m) + class_of_size(a.uni_n), s);
            if (have && (p.family == 0 || p.family == 1)) return launch_rt(a, p, s);
            if (uni && smm_fixed_available(a.uni_m, a.uni_n, a.uni_k))
                return launch_fixed(a, a.uni_m, static_cast<unsigned>(grid), s);
            return launch_rt(a, tuned_params(a), s);
        }
        case kSmmF64Fused: return launch_persistent(a, s);
        case kSmmF64Tuned: return launch_rt(a, tuned_params(a), s);
        default: set_error("unknown kernel variant %d", variant); return BSM_EINVAL;
    }
}

}  // namespace bsm
