// FP64 block products for uniform block sizes, one wavefront per quad of C
// blocks (2 x 2 group with a merged product list, built in quad.hip).
//
// Per entry k the wave stages the (up to) four operand blocks A(i_0, k),
// A(i_1, k), B(k, j_0), B(k, j_1) in LDS exactly as they sit in HBM, each read
// from HBM once, and multiplies every product (r, c) the entry holds.  The
// instruction and lane roles are those of the compile-time-shape kernel
// (V_MFMA_F64_4X4X4_4B_F64; lane = 16 x + 4 b + y, block b = 2 bh + bw owns
// the 4 x 4 tiles of row half bh and column half bw), but a lane's A values of
// row r serve both column blocks and its B values of column c both row
// blocks, so per k-step a lane reads 4H values from LDS for 4H^2 MFMAs
// instead of 2H for H^2.  Each C block's sum runs over its own products in
// ascending k exactly as in the one-block-per-wave kernels.  With two waves
// per quad each wave computes one row of the quad (two C blocks) and stages
// two of the four operand blocks.
#include <cstdlib>

#include "smm.h"

namespace bsm {

namespace {

template <int S>
struct QShape {
    static constexpr int B2 = S * S;
    static constexpr int MT = (S + 3) / 4, KS = MT, H = (MT + 1) / 2;
    static constexpr int KLAST = S - 4 * (KS - 1);   // valid x in the last k-step
    static constexpr int TAIL = 12 * S + 8;          // covers padded reads past the last block
    static constexpr int SIZE = 4 * B2 + TAIL;
    static constexpr int NV = (B2 + kWave - 1) / kWave;
};

__device__ inline int64_t quad_item(int64_t n_items) {
    const int64_t per = (n_items + kXcds - 1) / kXcds;
    return static_cast<int64_t>(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

__device__ inline double q_wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double q_wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// One entry's products for the rows [R0, R0 + NR) of the quad.  ALL: every
// operand present (no tests); otherwise the wave-uniform flags select the
// rows, columns and products.
template <int S, int NR, bool ALL>
__device__ inline void quad_step(const double *sm, int R0, int ra0, int rb0, bool klast_ok,
                                 const bool (&h)[4],
                                 double (&acc)[2 * NR][QShape<S>::H][QShape<S>::H]) {
    using Q = QShape<S>;
    constexpr int H = Q::H;
    bool ha[NR], hb[2];
#pragma unroll
    for (int r = 0; r < NR; ++r) ha[r] = ALL || h[R0 + r];
    hb[0] = ALL || h[2];
    hb[1] = ALL || h[3];
#pragma unroll
    for (int ks = 0; ks < Q::KS; ++ks) {
        double av[NR][H], bv[2][H];
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (ha[r]) {
#pragma unroll
                for (int t = 0; t < H; ++t)
                    av[r][t] = sm[(R0 + r) * Q::B2 + ra0 + 4 * t * S + 4 * ks];
            }
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (hb[c]) {
#pragma unroll
                for (int u = 0; u < H; ++u)
                    bv[c][u] = sm[(2 + c) * Q::B2 + rb0 + 4 * u + 4 * ks * S];
            }
        if (ks == Q::KS - 1 && Q::KLAST < 4) {
#pragma unroll
            for (int t = 0; t < H; ++t) {
#pragma unroll
                for (int r = 0; r < NR; ++r) av[r][t] = klast_ok ? av[r][t] : 0.0;
#pragma unroll
                for (int c = 0; c < 2; ++c) bv[c][t] = klast_ok ? bv[c][t] : 0.0;
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                if (ha[r] && hb[c]) {
#pragma unroll
                    for (int t = 0; t < H; ++t)
#pragma unroll
                        for (int u = 0; u < H; ++u)
                            acc[2 * r + c][t][u] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                                av[r][t], bv[c][u], acc[2 * r + c][t][u], 0, 0, 0);
                }
    }
}

// W wavefronts per quad: W = 1, the wave computes all four C blocks; W = 2,
// wave w computes the two C blocks of row w and stages A(i_w, k), B(k, j_w).
// WPE: the occupancy (waves per SIMD) the register allocation aims for.
template <int S, int W, int WPE>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_smm_f64_quad(SmmArgs a) {
    using Q = QShape<S>;
    constexpr int H = Q::H;
    constexpr int NR = (W == 1) ? 2 : 1;        // quad rows per wave
    constexpr int NZ = (W == 1) ? 4 : 2;        // operand blocks staged per wave
    __shared__ double sm[Q::SIZE];
    const int64_t item = quad_item(a.n_quads);
    if (item >= a.n_quads) return;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int R0 = (W == 1) ? 0 : wv;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3;
    const int bh = blk >> 1, bw = blk & 1;
    // staged block zz of this wave is quad operand zid(zz): A rows 0, 1 then B columns 0, 1
    auto zid = [&](int zz) { return (W == 1) ? zz : (zz == 0 ? wv : 2 + wv); };

    for (int e = 4 * Q::B2 + static_cast<int>(threadIdx.x); e < Q::SIZE; e += 64 * W) sm[e] = 0.0;
    const int ra0 = (4 * bh * H + y) * S + x;      // A(4 (bh H + t) + y, 4 ks + x)
    const int rb0 = x * S + 4 * bw * H + y;        // B(4 ks + x, 4 (bw H + u) + y)
    const bool klast_ok = x < Q::KLAST;

    double acc[2 * NR][H][H];
#pragma unroll
    for (int z = 0; z < 2 * NR; ++z)
#pragma unroll
        for (int t = 0; t < H; ++t)
#pragma unroll
            for (int u = 0; u < H; ++u) acc[z][t][u] = 0.0;

    const int64_t e0 = a.q_seg[item], e1 = a.q_seg[item + 1];
    double pv[NZ][Q::NV];
    int4 nxt = make_int4(-1, -1, -1, -1);
    auto prefetch = [&](int64_t e) {
        nxt = a.q_ent[e];
        const int id[4] = {nxt.x, nxt.y, nxt.z, nxt.w};
#pragma unroll
        for (int zz = 0; zz < NZ; ++zz) {
            const int z = zid(zz);
            if (id[z] >= 0) {
                const double *g = (z < 2 ? a.a_vals : a.b_vals) + static_cast<int64_t>(id[z]) * Q::B2;
#pragma unroll
                for (int q = 0; q < Q::NV; ++q)
                    if (q < Q::NV - 1 || lane + q * kWave < Q::B2) pv[zz][q] = g[lane + q * kWave];
            }
        }
    };
    if (e0 < e1) prefetch(e0);
    for (int64_t e = e0; e < e1; ++e) {
        const int4 cur = nxt;
        const bool h[4] = {cur.x >= 0, cur.y >= 0, cur.z >= 0, cur.w >= 0};
#pragma unroll
        for (int zz = 0; zz < NZ; ++zz) {
            const int z = zid(zz);
            if (h[z]) {
#pragma unroll
                for (int q = 0; q < Q::NV; ++q)
                    if (q < Q::NV - 1 || lane + q * kWave < Q::B2)
                        sm[z * Q::B2 + lane + q * kWave] = pv[zz][q];
            }
        }
        __syncthreads();
        if (e + 1 < e1) prefetch(e + 1);
        if (h[0] && h[1] && h[2] && h[3])
            quad_step<S, NR, true>(sm, R0, ra0, rb0, klast_ok, h, acc);
        else
            quad_step<S, NR, false>(sm, R0, ra0, rb0, klast_ok, h, acc);
        __syncthreads();
    }

#pragma unroll
    for (int zc = 0; zc < 2 * NR; ++zc) {
        const int64_t c = a.q_cblk[4 * item + 2 * R0 + zc];
        if (c < 0) continue;
        const int64_t co = a.c_blk_off[c];
        const double *cin = nullptr;
        if (a.cin_map) {
            const int64_t t = a.cin_map[c];
            if (t >= 0) cin = a.cin_vals + a.cin_blk_off[t];
        }
        double sq = 0.0, mx = 0.0;
#pragma unroll
        for (int t = 0; t < H; ++t)
#pragma unroll
            for (int u = 0; u < H; ++u) {
                const int row = 4 * (bh * H + t) + x, col = 4 * (bw * H + u) + y;
                if (row < S && col < S) {
                    double v = a.alpha * acc[zc][t][u];
                    if (cin) v += a.beta * cin[row * S + col];
                    a.c_vals[co + row * S + col] = v;
                    sq += v * v;
                    mx = fmax(mx, fabs(v));
                }
            }
        sq = q_wave_sum(sq);
        mx = q_wave_max(mx);
        if (lane == 0) {
            a.sq_out[c] = sq;
            a.mx_out[c] = mx;
            if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
        }
    }
}

}  // namespace

// Wavefronts per quad (1 or 2); BSM_QUAD_WAVES overrides the default.
static int quad_waves() {
    const char *e = getenv("BSM_QUAD_WAVES");
    return (e && atoi(e) == 1) ? 1 : 2;
}

bool smm_quad_available(int m, int n, int k) {
    return m == n && n == k && (m == 5 || m == 13 || m == 23);
}

int launch_quad(const SmmArgs &a, hipStream_t s) {
    if (a.n_quads <= 0) return BSM_OK;
    const int64_t per = (a.n_quads + kXcds - 1) / kXcds;
    const int64_t grid = per * kXcds;
    if (grid > (1ll << 31) - 1) {
        set_error("too many quads in one launch (%lld)", (long long)a.n_quads);
        return BSM_EINVAL;
    }
    const unsigned g = static_cast<unsigned>(grid);
    const int w = quad_waves();
    switch (a.uni_m) {
        case 5: k_smm_f64_quad<5, 1, 8><<<g, 64, 0, s>>>(a); break;
        case 13:
            if (w == 2) k_smm_f64_quad<13, 2, 4><<<g, 128, 0, s>>>(a);
            else k_smm_f64_quad<13, 1, 4><<<g, 64, 0, s>>>(a);
            break;
        case 23:
            if (w == 2) k_smm_f64_quad<23, 2, 3><<<g, 128, 0, s>>>(a);
            else k_smm_f64_quad<23, 1, 1><<<g, 64, 0, s>>>(a);
            break;
        default: set_error("no quad kernel for block size %d", a.uni_m); return BSM_EINVAL;
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
