// Tunable FP64 block-product kernels for run-time block shapes (m, n, k <= 32).
//
// The paper's GPU kernels are parametrised (threads per block, elements per
// thread, tiling, memory pattern) and an autotuner picks a parameter set for
// every (m, n, k) ("Batched execution" subsection).  The gfx950 kernels here
// expose three parameters:
//   FAM  matrix-core instruction: 0 = V_MFMA_F64_16X16X4_F64 (16 x 16 tiles),
//        1 = V_MFMA_F64_4X4X4_4B_F64 (4 x 4 tiles, four blocks per instruction);
//   WPG  C blocks per workgroup (1, 2, 4): one wavefront per C block, each
//        with its own LDS slice; waves never wait for each other;
//   PF   0 = load a product's operand blocks, then multiply; 1 = prefetch the
//        next product's blocks into registers while multiplying.
// All variants give the same sums in the same order (ascending k; inside a
// product the instruction's own k order), so they differ only in speed.
#include "smm.h"

namespace bsm {

typedef double d4 __attribute__((ext_vector_type(4)));

// Orders the LDS accesses of one wavefront: LDS operations of a wave are
// performed in order, so a compiler barrier with wavefront-scope fences is
// enough between a wave's own LDS writes and reads.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double rt_wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double rt_wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

template <int FAM, int T1, int T2, int WPG, int PF>
__global__ void __launch_bounds__(64 * WPG)
k_smm_f64_rt(SmmArgs a) {
    constexpr int kMaxM = FAM == 0 ? 16 * T1 : 8 * T1;
    constexpr int kMaxN = FAM == 0 ? 16 * T2 : 8 * T2;
    constexpr int NA = (kMaxM * kMaxBlock + kWave - 1) / kWave;
    constexpr int NB = (kMaxBlock * kMaxN + kWave - 1) / kWave;
    extern __shared__ double smem[];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    // workgroup g takes items WPG*g' .. WPG*g'+WPG-1 with g' XCD-contiguous
    const int64_t groups = (a.nC + WPG - 1) / WPG;
    const int64_t per = (groups + kXcds - 1) / kXcds;
    const int64_t g = static_cast<int64_t>(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int64_t item = g * WPG + wave;
    if (g >= groups || item >= a.nC) return;
    const int64_t c = a.worklist ? a.worklist[a.c0 + item] : a.c0 + item;
    double *sA = smem + static_cast<size_t>(wave) * (a.max_m * a.max_k + a.max_k * a.max_n);
    double *sB = sA + a.max_m * a.max_k;
    const int m = a.c_rbs[a.c_row[c]], n = a.c_cbs[a.c_col[c]];

    // FAM 0: lane = i + 16k (A), j + 16k (B); D(i,j) in lane j + 16*(i%4), reg i/4.
    // FAM 1: lane = 16x + 4b + y; A_b(i,k): x=k,y=i; B_b(k,j): x=k,y=j; D: x=i,y=j.
    const int r16 = lane & 15, kq = lane >> 4;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3, bh = blk >> 1, bw = blk & 1;
    const int t1n = FAM == 0 ? (m + 15) >> 4 : ((((m + 3) >> 2) + 1) >> 1);
    const int t2n = FAM == 0 ? (n + 15) >> 4 : ((((n + 3) >> 2) + 1) >> 1);

    d4 acc16[FAM == 0 ? T1 : 1][FAM == 0 ? T2 : 1];
    double acc4[FAM == 1 ? T1 : 1][FAM == 1 ? T2 : 1];
    if constexpr (FAM == 0) {
#pragma unroll
        for (int t = 0; t < T1; ++t)
#pragma unroll
            for (int u = 0; u < T2; ++u) acc16[t][u] = d4{0.0, 0.0, 0.0, 0.0};
    } else {
#pragma unroll
        for (int t = 0; t < T1; ++t)
#pragma unroll
            for (int u = 0; u < T2; ++u) acc4[t][u] = 0.0;
    }

    const int64_t p0 = a.seg[c - a.c0], p_end = a.seg[c - a.c0 + 1];
    double ra[PF ? NA : 1], rb[PF ? NB : 1];
    int k_next = 0;
    auto load_regs = [&](int64_t p) {
        const int32_t ta = a.stk_a[p];
        k_next = a.k_size[a.a_col_idx[ta]];
        const double *ga = a.a_vals + a.a_blk_off[ta];
        const double *gb = a.b_vals + a.b_blk_off[a.stk_b[p]];
        const int na = m * k_next, nb = k_next * n;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = lane + q * kWave;
            if (e < na) ra[q] = ga[e];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = lane + q * kWave;
            if (e < nb) rb[q] = gb[e];
        }
    };
    if constexpr (PF) {
        if (p0 < p_end) load_regs(p0);
    }
    for (int64_t p = p0; p < p_end; ++p) {
        int k;
        if constexpr (PF) {
            k = k_next;
#pragma unroll
            for (int q = 0; q < NA; ++q)
                if (lane + q * kWave < m * k) sA[lane + q * kWave] = ra[q];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (lane + q * kWave < k * n) sB[lane + q * kWave] = rb[q];
            wave_lds_sync();
            if (p + 1 < p_end) load_regs(p + 1);
        } else {
            const int32_t ta = a.stk_a[p];
            k = a.k_size[a.a_col_idx[ta]];
            const double *ga = a.a_vals + a.a_blk_off[ta];
            const double *gb = a.b_vals + a.b_blk_off[a.stk_b[p]];
            for (int e = lane; e < m * k; e += kWave) sA[e] = ga[e];
            for (int e = lane; e < k * n; e += kWave) sB[e] = gb[e];
            wave_lds_sync();
        }
        for (int ks = 0; ks < k; ks += 4) {
            if constexpr (FAM == 0) {
                const int kk = ks + kq;
                double av[T1], bv[T2];
#pragma unroll
                for (int t = 0; t < T1; ++t) {
                    const int r = 16 * t + r16;
                    av[t] = (r < m && kk < k) ? sA[r * k + kk] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < T2; ++u) {
                    const int cc = 16 * u + r16;
                    bv[u] = (kk < k && cc < n) ? sB[kk * n + cc] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < T1; ++t)
#pragma unroll
                    for (int u = 0; u < T2; ++u)
                        if (t < t1n && u < t2n)
                            acc16[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[u],
                                                                               acc16[t][u], 0, 0, 0);
            } else {
                const int kk = ks + x;
                double av[T1], bv[T2];
#pragma unroll
                for (int t = 0; t < T1; ++t) {
                    const int r = 4 * (bh * t1n + t) + y;
                    av[t] = (t < t1n && r < m && kk < k) ? sA[r * k + kk] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < T2; ++u) {
                    const int cc = 4 * (bw * t2n + u) + y;
                    bv[u] = (u < t2n && cc < n && kk < k) ? sB[kk * n + cc] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < T1; ++t)
#pragma unroll
                    for (int u = 0; u < T2; ++u)
                        if (t < t1n && u < t2n)
                            acc4[t][u] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[t], bv[u],
                                                                           acc4[t][u], 0, 0, 0);
            }
        }
        wave_lds_sync();
    }

    const int64_t co = a.c_blk_off[c];
    const double *cin = nullptr;
    if (a.cin_map) {
        const int64_t t = a.cin_map[c];
        if (t >= 0) cin = a.cin_vals + a.cin_blk_off[t];
    }
    double sq = 0.0, mx = 0.0;
    auto emit = [&](int row, int col, double s) {
        if (row < m && col < n) {
            double v = a.alpha * s;
            if (cin) v += a.beta * cin[row * n + col];
            a.c_vals[co + row * n + col] = v;
            sq += v * v;
            mx = fmax(mx, fabs(v));
        }
    };
    if constexpr (FAM == 0) {
#pragma unroll
        for (int t = 0; t < T1; ++t)
#pragma unroll
            for (int u = 0; u < T2; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    emit(16 * t + 4 * q + kq, 16 * u + r16, acc16[t][u][q]);
    } else {
#pragma unroll
        for (int t = 0; t < T1; ++t)
#pragma unroll
            for (int u = 0; u < T2; ++u)
                if (t < t1n && u < t2n) emit(4 * (bh * t1n + t) + x, 4 * (bw * t2n + u) + y, acc4[t][u]);
    }
    sq = rt_wave_sum(sq);
    mx = rt_wave_max(mx);
    if (lane == 0) {
        a.sq_out[c] = sq;
        a.mx_out[c] = mx;
        if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
    }
}

template <int FAM, int T1, int T2>
static int launch_rt_fam(const SmmArgs &a, int wpg, int pf, hipStream_t s) {
    const int64_t groups = (a.nC + wpg - 1) / wpg;
    const int64_t per = (groups + kXcds - 1) / kXcds;
    const unsigned grid = static_cast<unsigned>(per * kXcds);
    const size_t lds = sizeof(double) * static_cast<size_t>(wpg) *
                       (static_cast<size_t>(a.max_m) * a.max_k + static_cast<size_t>(a.max_k) * a.max_n);
#define BSM_RT(W, P) BSM_LAUNCH((k_smm_f64_rt<FAM, T1, T2, W, P>), grid, 64 * W, lds, s)(a)
    if (wpg == 1) { if (pf) BSM_RT(1, 1); else BSM_RT(1, 0); }
    else if (wpg == 2) { if (pf) BSM_RT(2, 1); else BSM_RT(2, 0); }
    else { if (pf) BSM_RT(4, 1); else BSM_RT(4, 0); }
#undef BSM_RT
    note_kernelf("k_smm_f64_rt<%d, %d, %d, %d, %d>", FAM, T1, T2, wpg == 2 || wpg == 4 ? wpg : 1, pf);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int launch_rt(const SmmArgs &a, const SmmParams &prm, hipStream_t s) {
    if (a.nC <= 0) return BSM_OK;
    if (a.max_m > kMaxBlock || a.max_n > kMaxBlock || a.max_k > kMaxBlock) {
        set_error("block sizes above %d", kMaxBlock);
        return BSM_EINVAL;
    }
    const int wpg = (prm.wpg == 2 || prm.wpg == 4) ? prm.wpg : 1;
    const int pf = prm.prefetch ? 1 : 0;
    if (prm.family == 0) {
        const int t1 = a.max_m <= 16 ? 1 : 2, t2 = a.max_n <= 16 ? 1 : 2;
        if (t1 == 1 && t2 == 1) return launch_rt_fam<0, 1, 1>(a, wpg, pf, s);
        if (t1 == 1) return launch_rt_fam<0, 1, 2>(a, wpg, pf, s);
        if (t2 == 1) return launch_rt_fam<0, 2, 1>(a, wpg, pf, s);
        return launch_rt_fam<0, 2, 2>(a, wpg, pf, s);
    }
    const int t = std::max((((a.max_m + 3) / 4) + 1) / 2, (((a.max_n + 3) / 4) + 1) / 2);
    if (t <= 1) return launch_rt_fam<1, 1, 1>(a, wpg, pf, s);
    if (t <= 2) return launch_rt_fam<1, 2, 2>(a, wpg, pf, s);
    if (t <= 3) return launch_rt_fam<1, 3, 3>(a, wpg, pf, s);
    return launch_rt_fam<1, 4, 4>(a, wpg, pf, s);
}

}  // namespace bsm
