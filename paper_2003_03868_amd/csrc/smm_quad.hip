// FP64 block products for uniform block sizes, one workgroup per GR x GC
// group of C blocks (2 x 2: quads, the default; 4 x 4 and 4 x 2 on request)
// with a merged product list (built in quad.hip).
//
// Per entry k the workgroup stages the (up to) GR + GC operand blocks
// A(i_r, k), B(k, j_c) in LDS exactly as they sit in HBM, each read from HBM
// once, and multiplies every product (r, c) the entry holds; each C block's
// sum runs over its own products in ascending k exactly as in the
// one-block-per-wave kernels, with the same instructions, so the results are
// the same bits.  Instruction and lane roles are those of the
// compile-time-shape kernel (V_MFMA_F64_4X4X4_4B_F64; lane = 16 x + 4 b + y,
// block b = 2 bh + bw owns the 4 x 4 tiles of row half bh and column half
// bw).  With W waves per group, a wave computes GR GC / W of the C blocks
// (an NR x NC patch) and stages operands wv, wv + W, ... (quads: W = 4, one
// each, the fastest form on the sign workload; W = 1: one wave reads each A
// value once for two column blocks and each B value once for two row
// blocks).  Operands of the next entry are prefetched into registers; entry
// indices are staged through LDS in chunks, so no load waits on another load
// of the same iteration.
#include <cstdlib>
#include <type_traits>

#include "smm.h"

namespace bsm {

namespace {

template <int S>
struct QShape {
    static constexpr int B2 = S * S;
    static constexpr int MT = (S + 3) / 4, KS = MT, H = (MT + 1) / 2;
    static constexpr int KLAST = S - 4 * (KS - 1);   // valid x in the last k-step
    static constexpr int TAIL = 12 * S + 8;          // covers padded reads past the last block
    static constexpr int NV = (B2 + kWave - 1) / kWave;
};

// Entry indices read from LDS are the same in every lane; saying so keeps
// the operand tests wave-uniform (scalar branches, no exec-mask merges).
__device__ inline int4 uniform4(int4 v) {
    return make_int4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                     __builtin_amdgcn_readfirstlane(v.z), __builtin_amdgcn_readfirstlane(v.w));
}

// Work item of this workgroup: the items form kXcds contiguous ranges, range
// x for the workgroups blockIdx.x % kXcds = x (which run on one XCD); n_items
// for a workgroup past the last range.
__device__ inline int64_t quad_item(int64_t n_items) {
    const int64_t per = (n_items + kXcds - 1) / kXcds;
    if (static_cast<int64_t>(blockIdx.x / kXcds) >= per) return n_items;
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

// One entry's products of the wave: product (r, c) (rows [R0, R0 + NR),
// columns [C0, C0 + NC) of the group) is done when bit NC r + c of PM is set.
// PM is a compile-time constant, so the k loop holds no tests; A rows and B
// columns no product uses are not read.
template <int S, int GR, int NR, int NC, unsigned PM>
__device__ inline void quad_step(const double *sm, int R0, int C0, int ra0, int rb0,
                                 bool klast_ok,
                                 double (&acc)[NR * NC][QShape<S>::H][QShape<S>::H]) {
    using Q = QShape<S>;
    constexpr int H = Q::H;
#pragma unroll
    for (int ks = 0; ks < Q::KS; ++ks) {
        if (GR == 4) __builtin_amdgcn_sched_barrier(0);
        double av[NR][H], bv[NC][H];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            constexpr unsigned rowbits = (1u << NC) - 1u;
            if ((PM >> (NC * r)) & rowbits) {
#pragma unroll
                for (int t = 0; t < H; ++t) {
                    const double v = sm[(R0 + r) * Q::B2 + ra0 + 4 * t * S + 4 * ks];
                    av[r][t] = (ks == Q::KS - 1 && Q::KLAST < 4 && !klast_ok) ? 0.0 : v;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            unsigned colbits = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r) colbits |= 1u << (NC * r + c);
            if (PM & colbits) {
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const double v = sm[(GR + C0 + c) * Q::B2 + rb0 + 4 * u + 4 * ks * S];
                    bv[c][u] = (ks == Q::KS - 1 && Q::KLAST < 4 && !klast_ok) ? 0.0 : v;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if ((PM >> (NC * r + c)) & 1u) {
#pragma unroll
                    for (int t = 0; t < H; ++t)
#pragma unroll
                        for (int u = 0; u < H; ++u)
                            acc[NC * r + c][t][u] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                                av[r][t], bv[c][u], acc[NC * r + c][t][u], 0, 0, 0);
                }
    }
}

// The wave's products of an entry with operand flags hm (bit z: operand z
// present): dispatch on the wave's product mask to a compile-time variant.
template <int S, int GR, int GC, int NR, int NC>
__device__ inline void quad_entry(const double *sm, int R0, int C0, int ra0, int rb0,
                                  bool klast_ok, unsigned hm, unsigned gm,
                                  double (&acc)[NR * NC][QShape<S>::H][QShape<S>::H]) {
    // gm: the entry's product mask over the group (bit GC r + c; all ones
    // without screening)
    unsigned pm = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (((hm >> (R0 + r)) & 1u) && ((hm >> (GR + C0 + c)) & 1u) &&
                ((gm >> (GC * (R0 + r) + C0 + c)) & 1u))
                pm |= 1u << (NC * r + c);
#define BSM_QS(M) \
    case M: quad_step<S, GR, NR, NC, (M)>(sm, R0, C0, ra0, rb0, klast_ok, acc); break;
    if (NR * NC == 1) {
        if (pm) quad_step<S, GR, NR, NC, 1u>(sm, R0, C0, ra0, rb0, klast_ok, acc);
    } else if (NR * NC == 2) {
        switch (pm) { BSM_QS(1u) BSM_QS(2u) BSM_QS(3u) default: break; }
    } else {
        switch (pm) {
            BSM_QS(1u) BSM_QS(2u) BSM_QS(3u) BSM_QS(4u) BSM_QS(5u) BSM_QS(6u) BSM_QS(7u)
            BSM_QS(8u) BSM_QS(9u) BSM_QS(10u) BSM_QS(11u) BSM_QS(12u) BSM_QS(13u) BSM_QS(14u)
            BSM_QS(15u)
            default: break;
        }
    }
#undef BSM_QS
}

// alpha * sum + beta * C_in for the wave's C blocks of group `item`, with the
// blocks' filter norms.
template <int S, int GR, int GC, int NR, int NC>
__device__ inline void quad_store(const SmmArgs &a, int64_t item, int R0, int C0, int lane,
                                  const double (&acc)[NR * NC][QShape<S>::H][QShape<S>::H]) {
    constexpr int H = QShape<S>::H;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3;
    const int bh = blk >> 1, bw = blk & 1;
#pragma unroll
    for (int zc = 0; zc < NR * NC; ++zc) {
        const int64_t c = a.q_cblk[GR * GC * item + GC * (R0 + zc / NC) + C0 + zc % NC];
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

// W wavefronts per group.  Quads: W = 1, the wave computes all four C
// blocks; W = 2, wave w computes the two C blocks of row w and stages
// A(i_w, k), B(k, j_w); W = 4, wave w computes C block (w / 2, w % 2) and
// stages operand w.  Groups of sixteen: W = 16, wave w computes C block
// (w / 4, w % 4), and waves w and w + 8 stage the two halves of operand
// w % 8 (with eight waves, two C blocks each, the register demand spills).
// 4 x 2 groups: W = 8, wave w computes C block (w / 2, w % 2); waves 0..5
// stage the four A and two B blocks.
// WPE: the occupancy (waves per SIMD) the register allocation aims for.
// MK: entries carry product masks (norm screening, a.q_pm).
template <int S, int GR, int GC, int W, int WPE, int EPS, bool MK = false>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_smm_f64_quad(SmmArgs a) {
    using Q = QShape<S>;
    constexpr int H = Q::H;
    constexpr int NPW = GR * GC / W;            // C blocks per wave
    constexpr int NC = NPW < GC ? NPW : GC;     // group columns per wave
    constexpr int NR = NPW / NC;                // group rows per wave
    constexpr int NOP = GR + GC;                // operand blocks per entry
    constexpr int WPO = W > NOP ? W / NOP : 1;  // waves sharing the staging of one block
    constexpr int NZ = W > NOP ? 1 : NOP / W;   // operand blocks (or parts) staged per wave
    constexpr int NVP = (Q::NV + WPO - 1) / WPO;  // register slots of one staged part
    constexpr int NE = (NOP + 3) / 4;           // int4 per entry
    constexpr int SLOT = NOP * Q::B2;           // LDS doubles of one staged entry
    static_assert(NE <= 2 && GC % NC == 0, "group shapes up to 4 x 4");
    static_assert(NR * NC * W == GR * GC, "waves must tile the group");
    static_assert(W > NOP || NOP % W == 0, "operands must split evenly over the waves");
    __shared__ double sm[EPS * SLOT + Q::TAIL];
    const int64_t n_items = a.n_quads_dev ? *a.n_quads_dev : a.n_quads;
    const int64_t it = quad_item(n_items);
    if (it >= n_items) return;
    const int64_t item = a.q_order ? a.q_order[it] : it;
    const int lane = threadIdx.x % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));  // wave-uniform
    const int R0 = (wv / (GC / NC)) * NR;
    const int C0 = (wv % (GC / NC)) * NC;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3;
    const int bh = blk >> 1, bw = blk & 1;
    // staged block zz of this wave is entry operand wv + W zz (A rows 0 .. GR-1,
    // then B columns); with more waves than operands, wave wv < WPO NOP stages
    // part wv / NOP (slots [part NVP, part NVP + NVP)) of operand wv % NOP and
    // the other waves stage nothing
    static_assert(WPO <= 2, "a block is staged by one or two waves");
    auto zid = [&](int zz) { return W > NOP ? wv % NOP : wv + W * zz; };
    const int part = W > NOP ? wv / NOP : 0;
    const bool stager = W <= NOP || wv < WPO * NOP;
    // element lane + 64 (P NVP + v) of a block exists (compile-time but for the last slot)
    auto has = [&](auto P, int v) {
        constexpr int p0 = decltype(P)::value * NVP;
        return p0 + v < Q::NV - 1 || (p0 + v == Q::NV - 1 && lane + (p0 + v) * kWave < Q::B2);
    };
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    auto pick = [](const int4 (&v)[NE], int z) {
        const int4 e = (z < 4) ? v[0] : v[NE - 1];   // selects, not a run-time array index
        const int c = z & 3;
        return c == 0 ? e.x : c == 1 ? e.y : c == 2 ? e.z : e.w;
    };

    for (int e = EPS * SLOT + static_cast<int>(threadIdx.x); e < EPS * SLOT + Q::TAIL; e += 64 * W)
        sm[e] = 0.0;
    const int ra0 = (4 * bh * H + y) * S + x;      // A(4 (bh H + t) + y, 4 ks + x)
    const int rb0 = x * S + 4 * bw * H + y;        // B(4 ks + x, 4 (bw H + u) + y)
    const bool klast_ok = x < Q::KLAST;

    double acc[NR * NC][H][H];
#pragma unroll
    for (int z = 0; z < NR * NC; ++z)
#pragma unroll
        for (int t = 0; t < H; ++t)
#pragma unroll
            for (int u = 0; u < H; ++u) acc[z][t][u] = 0.0;

    // Pipeline: while the EPS entries of a stage are multiplied, the operand
    // blocks of the next stage are in flight to registers.  The entry indices
    // come from LDS, where wave 0 stores them in chunks of kEntryChunk
    // (double-buffered; the next chunk waits in registers), so no global load
    // waits on another global load issued in the same iteration.
    constexpr int kEntryChunk = 64;
    static_assert(kEntryChunk % EPS == 0, "stages must not straddle index chunks");
    __shared__ int4 ebuf[2][kEntryChunk][NE];
    __shared__ int32_t pbuf[2][MK ? kEntryChunk : 1];     // product masks of the chunk
    const int64_t e0 = a.q_seg[item], ne = a.q_seg[item + 1] - e0;
    double pv[EPS][NZ][NVP];
    auto load_blocks = [&](const int4 (&en)[NE], double (&p)[NZ][NVP]) {
#pragma unroll
        for (int zz = 0; zz < NZ; ++zz) {
            const int z = zid(zz);
            const int id = stager ? pick(en, z) : -1;
            if (id >= 0) {
                const double *g = (z < GR ? a.a_vals : a.b_vals) + static_cast<int64_t>(id) * Q::B2;
                auto ld = [&](auto P) {
                    constexpr int p0 = decltype(P)::value * NVP;
#pragma unroll
                    for (int q = 0; q < NVP; ++q)
                        if (has(P, q)) p[zz][q] = g[lane + (p0 + q) * kWave];
                };
                if (WPO == 1 || part == 0) ld(P0{}); else ld(P1{});
            }
        }
    };
    auto flags = [](const int4 (&c)[NE]) {
        unsigned f = 0;
#pragma unroll
        for (int h = 0; h < NE; ++h)
            f |= ((c[h].x >= 0 ? 1u : 0u) | (c[h].y >= 0 ? 2u : 0u) | (c[h].z >= 0 ? 4u : 0u) |
                  (c[h].w >= 0 ? 8u : 0u)) << (4 * h);
        // bit z: operand z present (A rows 0 .. GR-1, then B columns)
        return f;
    };
    auto fetch = [&](int64_t t, int4 (&out)[NE], unsigned &gm) {
#pragma unroll
        for (int h = 0; h < NE; ++h)
            out[h] = (t < ne) ? uniform4(ebuf[(t / kEntryChunk) & 1][t % kEntryChunk][h])
                              : make_int4(-1, -1, -1, -1);
        gm = ~0u;
        if (MK && t < ne)
            gm = static_cast<unsigned>(
                __builtin_amdgcn_readfirstlane(pbuf[(t / kEntryChunk) & 1][t % kEntryChunk]));
    };
    int4 creg[NE];                             // wave 0: entry e0 + 64 c + lane of the next chunk
    int32_t cpm = 0;                           // and its product mask
#pragma unroll
    for (int h = 0; h < NE; ++h) creg[h] = make_int4(-1, -1, -1, -1);
    if (wv == 0) {
#pragma unroll
        for (int h = 0; h < NE; ++h) {
            if (lane < ne) ebuf[0][lane][h] = a.q_ent[NE * (e0 + lane) + h];
            if (kEntryChunk + lane < ne) creg[h] = a.q_ent[NE * (e0 + kEntryChunk + lane) + h];
        }
        if (MK) {
            if (lane < ne) pbuf[0][lane] = a.q_pm[e0 + lane];
            if (kEntryChunk + lane < ne) cpm = a.q_pm[e0 + kEntryChunk + lane];
        }
    }
    __syncthreads();
    int4 nxt[EPS][NE];
    unsigned ngm[EPS];
#pragma unroll
    for (int q = 0; q < EPS; ++q) {
        fetch(q, nxt[q], ngm[q]);
        load_blocks(nxt[q], pv[q]);
    }
    for (int64_t t = 0; t < ne; t += EPS) {
        unsigned hm[EPS], gm[EPS];
#pragma unroll
        for (int q = 0; q < EPS; ++q) {
            hm[q] = flags(nxt[q]);
            gm[q] = ngm[q];
#pragma unroll
            for (int zz = 0; zz < NZ; ++zz) {
                const int z = zid(zz);
                if (stager && ((hm[q] >> z) & 1u)) {
                    auto st = [&](auto P) {
                        constexpr int p0 = decltype(P)::value * NVP;
#pragma unroll
                        for (int v = 0; v < NVP; ++v)
                            if (has(P, v)) sm[q * SLOT + z * Q::B2 + lane + (p0 + v) * kWave] = pv[q][zz][v];
                    };
                    if (WPO == 1 || part == 0) st(P0{}); else st(P1{});
                }
            }
        }
        const int64_t t1 = t + EPS;
        if ((t1 % kEntryChunk) == 0 && t1 < ne && wv == 0) {
            // entering chunk t1 / 64: its indices (loaded a chunk ago) go to
            // LDS, the chunk after it is fetched into registers
#pragma unroll
            for (int h = 0; h < NE; ++h) {
                ebuf[(t1 / kEntryChunk) & 1][lane][h] = creg[h];
                if (t1 + kEntryChunk + lane < ne) creg[h] = a.q_ent[NE * (e0 + t1 + kEntryChunk + lane) + h];
            }
            if (MK) {
                pbuf[(t1 / kEntryChunk) & 1][lane] = cpm;
                if (t1 + kEntryChunk + lane < ne) cpm = a.q_pm[e0 + t1 + kEntryChunk + lane];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPS; ++q) {
            fetch(t1 + q, nxt[q], ngm[q]);
            load_blocks(nxt[q], pv[q]);
        }
#pragma unroll
        for (int q = 0; q < EPS; ++q)
            quad_entry<S, GR, GC, NR, NC>(sm + q * SLOT, R0, C0, ra0, rb0, klast_ok, hm[q], gm[q],
                                          acc);
        __syncthreads();
    }

    quad_store<S, GR, GC, NR, NC>(a, item, R0, C0, lane, acc);
}

}  // namespace

// Wavefronts per quad (1, 2 or 4, measured best 4; groups of sixteen always
// use 16); BSM_QUAD_WAVES overrides the default.
static int quad_waves() {
    const char *e = getenv("BSM_QUAD_WAVES");
    const int w = e ? atoi(e) : 4;
    return (w == 1 || w == 2) ? w : 4;
}

// Entries staged per barrier pair (1 or 2, quads only); BSM_QUAD_STAGE overrides the default.
static int quad_stage() {
    const char *e = getenv("BSM_QUAD_STAGE");
    return (e && atoi(e) == 2) ? 2 : 1;
}

bool smm_quad_available(int m, int n, int k) {
    return m == n && n == k && (m == 5 || m == 6 || m == 13 || m == 23 || m == 26 || m == 32);
}

void quad_shape(int m, int *gr, int *gc) {
    const char *e = getenv("BSM_QUAD_GROUP");
    const int g = e ? atoi(e) : 2;
    *gr = *gc = 2;
    if (m == 5 || m == 6) return;
    if (g == 4) { *gr = 4; *gc = 4; }
    else if (g == 42 && m == 23) { *gr = 4; *gc = 2; }
}

int launch_quad(const SmmArgs &a, hipStream_t s) {
    if (a.prec != BSM_FP64) return launch_lowp_quad(a, s);
    if (a.n_quads <= 0) return BSM_OK;
    const int64_t per = (a.n_quads + kXcds - 1) / kXcds;
    const int64_t grid = per * kXcds;
    if (grid > (1ll << 31) - 1) {
        set_error("too many quads in one launch (%lld)", (long long)a.n_quads);
        return BSM_EINVAL;
    }
    const unsigned g = static_cast<unsigned>(grid);
    const int w = quad_waves(), eps = quad_stage();
    if (a.q_pm) {
        // product masks (norm screening): quads with four waves (sizes 5, 6: one)
        if (a.q_gr != 2 || a.q_gc != 2) { set_error("internal: masked groups are quads"); return BSM_EINVAL; }
        switch (a.uni_m) {
            case 5: BSM_LAUNCH((k_smm_f64_quad<5, 2, 2, 1, 6, 1, true>), g, 64, 0, s)(a); break;
            case 6: BSM_LAUNCH((k_smm_f64_quad<6, 2, 2, 1, 6, 1, true>), g, 64, 0, s)(a); break;
            case 13: BSM_LAUNCH((k_smm_f64_quad<13, 2, 2, 4, 6, 1, true>), g, 256, 0, s)(a); break;
            case 23: BSM_LAUNCH((k_smm_f64_quad<23, 2, 2, 4, 5, 1, true>), g, 256, 0, s)(a); break;
            case 26: BSM_LAUNCH((k_smm_f64_quad<26, 2, 2, 4, 4, 1, true>), g, 256, 0, s)(a); break;
            case 32: BSM_LAUNCH((k_smm_f64_quad<32, 2, 2, 4, 4, 1, true>), g, 256, 0, s)(a); break;
            default: set_error("no quad kernel for block size %d", a.uni_m); return BSM_EINVAL;
        }
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
    if (a.q_gr == 4 && a.q_gc == 2 && a.uni_m == 23) {
        BSM_LAUNCH((k_smm_f64_quad<23, 4, 2, 8, 6, 1>), g, 512, 0, s)(a);
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
    if (a.q_gr == 4 && a.q_gc == 4) {
        switch (a.uni_m) {
            case 13: BSM_LAUNCH((k_smm_f64_quad<13, 4, 4, 16, 8, 1>), g, 1024, 0, s)(a); break;
            case 23: BSM_LAUNCH((k_smm_f64_quad<23, 4, 4, 16, 8, 1>), g, 1024, 0, s)(a); break;
            case 26: BSM_LAUNCH((k_smm_f64_quad<26, 4, 4, 16, 4, 1>), g, 1024, 0, s)(a); break;
            case 32: BSM_LAUNCH((k_smm_f64_quad<32, 4, 4, 16, 4, 1>), g, 1024, 0, s)(a); break;
            default: set_error("no group-of-sixteen kernel for block size %d", a.uni_m); return BSM_EINVAL;
        }
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
    if (a.q_gr != 2 || a.q_gc != 2) {
        set_error("internal: no %d x %d group kernel for block size %d", a.q_gr, a.q_gc, a.uni_m);
        return BSM_EINVAL;
    }
    switch (a.uni_m) {
        case 5: BSM_LAUNCH((k_smm_f64_quad<5, 2, 2, 1, 8, 1>), g, 64, 0, s)(a); break;
        case 6: BSM_LAUNCH((k_smm_f64_quad<6, 2, 2, 1, 8, 1>), g, 64, 0, s)(a); break;
        case 13:
            if (w == 4) BSM_LAUNCH((k_smm_f64_quad<13, 2, 2, 4, 6, 1>), g, 256, 0, s)(a);
            else if (w == 2) BSM_LAUNCH((k_smm_f64_quad<13, 2, 2, 2, 4, 1>), g, 128, 0, s)(a);
            else BSM_LAUNCH((k_smm_f64_quad<13, 2, 2, 1, 4, 1>), g, 64, 0, s)(a);
            break;
        case 23:
            if (w == 4 && eps == 2) BSM_LAUNCH((k_smm_f64_quad<23, 2, 2, 4, 4, 2>), g, 256, 0, s)(a);
            else if (w == 4) BSM_LAUNCH((k_smm_f64_quad<23, 2, 2, 4, 6, 1>), g, 256, 0, s)(a);   // 6 waves/SIMD: 1% faster than 5
            else if (w == 2) BSM_LAUNCH((k_smm_f64_quad<23, 2, 2, 2, 3, 1>), g, 128, 0, s)(a);
            else BSM_LAUNCH((k_smm_f64_quad<23, 2, 2, 1, 1, 1>), g, 64, 0, s)(a);
            break;
        case 26: BSM_LAUNCH((k_smm_f64_quad<26, 2, 2, 4, 4, 1>), g, 256, 0, s)(a); break;
        case 32: BSM_LAUNCH((k_smm_f64_quad<32, 2, 2, 4, 4, 1>), g, 256, 0, s)(a); break;
        default: set_error("no quad kernel for block size %d", a.uni_m); return BSM_EINVAL;
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
