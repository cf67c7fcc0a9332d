// Reduced-precision block products (the approximate-computing direction of
// the paper: lower or mixed precision where FP64 accuracy is not needed,
// "Approximate Computing" section and the DBCSR "Outlook").
//
// Two forms, both accumulating each block product in FP32 on the matrix
// cores and adding it into an FP64 accumulator per C block (so the error of
// one product does not grow with the length of the product stack); the
// result, its norms and the filter stay FP64:
//
//  * FP32:       operands rounded to FP32; V_MFMA_F32_16X16X4_F32.
//  * split-BF16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (both
//                round-to-nearest-even); A*B ~ lo*hi + hi*lo + hi*hi with
//                V_MFMA_F32_32X32X16_BF16 (the lo*lo term is dropped).
//                Each operand keeps about 17 significant bits.
//  * three-term split-BF16: x = hi + mid + lo, each part the RNE bf16 of
//                what the previous parts leave; with |mid| <= 2^-9 |x| and
//                |lo| <= 2^-18 |x| the products are kept down to size
//                2^-18 of hi*hi: mid*mid + hi*lo + lo*hi + mid*hi + hi*mid
//                + hi*hi (small terms first).  About 26 bits per operand,
//                so the FP32 accumulation sets the error, as in FP32 mode.
//
// Operands are packed once per multiply: one 32-bit word per element (the
// FP32 bits, or hi << 16 | lo), and for the three-term split hi << 16 | mid
// followed by an array of the lo parts (uint16).  Kernels exist for uniform
// block sizes (compile-time shapes, up to 32).
#include "smm.h"

namespace bsm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// --------------------------------------------------------------- packing

// Round-to-odd double -> float followed by round-to-nearest-even float ->
// bf16 gives the correctly rounded (RNE) bf16 of the double: the float keeps
// 24 significant bits, more than the 8 + 2 the second rounding needs.
__device__ inline uint32_t bf16_rne(double x) {
    float t = __double2float_rz(x);
    if (static_cast<double>(t) != x) t = __uint_as_float(__float_as_uint(t) | 1u);
    uint32_t u = __float_as_uint(t);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ inline double bf16_to_double(uint32_t h) {
    return static_cast<double>(__uint_as_float(h << 16));
}

__global__ void k_pack_lowp(const double *v, int64_t n, uint32_t *out, int prec) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = v[i];
    if (prec == BSM_FP32) {
        out[i] = __float_as_uint(__double2float_rn(x));
    } else {
        // x - hi and r - mid are exact in FP64 (the parts are RNE roundings
        // of the value they are subtracted from, far above its last bit)
        const uint32_t hi = bf16_rne(x);
        const double r = x - bf16_to_double(hi);
        const uint32_t nxt = bf16_rne(r);
        out[i] = (hi << 16) | nxt;
        if (prec == BSM_SPLIT_BF16X3) {
            const uint32_t lo = bf16_rne(r - bf16_to_double(nxt));
            reinterpret_cast<unsigned short *>(out + n)[i] = static_cast<unsigned short>(lo);
        }
    }
}

int pack_lowp(const double *v, int64_t n, uint32_t *out, int prec, hipStream_t s) {
    if (n == 0) return BSM_OK;
    k_pack_lowp<<<grid_for(n, 256), 256, 0, s>>>(v, n, out, prec);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

__device__ inline int64_t lp_item(int64_t n_items) {
    const int64_t per = (n_items + kXcds - 1) / kXcds;
    return static_cast<int64_t>(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

__device__ inline double lp_wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double lp_wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Epilogue shared by both forms: out(row, col) for the lane's 16 slots.
template <int M, int N, class RowCol>
__device__ inline void lp_store(const SmmArgs &a, int64_t c, const double (&acc)[16],
                                RowCol rc) {
    const int64_t co = a.c_blk_off[c];
    const double *cin = nullptr;
    if (a.cin_map) {
        const int64_t t = a.cin_map[c];
        if (t >= 0) cin = a.cin_vals + a.cin_blk_off[t];
    }
    double sq = 0.0, mx = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        int row, col;
        rc(q, row, col);
        if (row < M && col < N) {
            double v = a.alpha * acc[q];
            if (cin) v += a.beta * cin[row * N + col];
            a.c_vals[co + row * N + col] = v;
            sq += v * v;
            mx = fmax(mx, fabs(v));
        }
    }
    sq = lp_wave_sum(sq);
    mx = lp_wave_max(mx);
    if (threadIdx.x == 0) {
        a.sq_out[c] = sq;
        a.mx_out[c] = mx;
        if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
    }
}

// ------------------------------------------------------------ split-BF16
// One wavefront per C block, the block padded to one 32 x 32 tile.
// LDS: A_hi, A_lo as [32][LDK] and B_hi^T, B_lo^T as [32][LDK] (bf16), so
// each lane reads its 8 consecutive k values with one 16-byte load.
// Lane layout of V_MFMA_F32_32X32X16_BF16 (measured on gfx950):
// A(i,k): lane i + 32*(k/8), element k%8; B(k,j): lane j + 32*(k/8),
// element k%8; D(i,j): lane j + 32*((i/4)%2), register 4*(i/8) + i%4.
// One split block product over KS k steps of 16, added into the FP64
// accumulator.  T = 2: LDS planes hi, lo of A then of B, per k step
// lo*hi + hi*lo + hi*hi.  T = 3: planes hi, mid, lo; first every correction
// term (mid*mid, lo*hi, hi*lo, mid*hi, hi*mid) of all k steps, then hi*hi of
// all k steps, so that the small terms are summed while the FP32 sum is
// still small and are not rounded to the precision of hi*hi.
template <int T, int KS, int LDK, int PLANE>
__device__ inline void bf16_split_product(const unsigned short *as, const unsigned short *bs,
                                          int base, double (&acc)[16]) {
    auto ld = [&](const unsigned short *p, int q, int ks) {
        return __builtin_bit_cast(bf8, *reinterpret_cast<const us8 *>(p + q * PLANE + base + 16 * ks));
    };
    f16v part = {};
    if (T == 3) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf8 ah = ld(as, 0, ks), am = ld(as, 1, ks), al = ld(as, 2, ks);
            const bf8 bh = ld(bs, 0, ks), bm = ld(bs, 1, ks), bl = ld(bs, 2, ks);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, part, 0, 0, 0);
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld(as, 0, ks), ld(bs, 0, ks), part, 0, 0, 0);
    } else {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf8 ah = ld(as, 0, ks), al = ld(as, 1, ks), bh = ld(bs, 0, ks), bl = ld(bs, 1, ks);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, part, 0, 0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] += static_cast<double>(part[q]);
}

template <int M, int N, int K, int T>
__global__ void __launch_bounds__(64)
k_smm_bf16x3(SmmArgs a) {
    constexpr int LDK = 40;                         // 80-byte rows: conflict-free 16 B reads
    constexpr int PLANE = 32 * LDK;
    constexpr int KS = (K + 15) / 16;
    constexpr int NA = (M * K + kWave - 1) / kWave, NB = (K * N + kWave - 1) / kWave;
    __shared__ __attribute__((aligned(16))) unsigned short sm[2 * T * PLANE];
    unsigned short *as = sm, *bs = sm + T * PLANE;
    const int64_t item = lp_item(a.nC);
    if (item >= a.nC) return;
    const int lane = threadIdx.x;
    const int64_t c = a.worklist ? a.worklist[a.c0 + item] : a.c0 + item;
    for (int e = lane; e < 2 * T * PLANE; e += kWave) sm[e] = 0;
    const unsigned short *alo3 = reinterpret_cast<const unsigned short *>(a.a_pk + a.a_pk_n);
    const unsigned short *blo3 = reinterpret_cast<const unsigned short *>(a.b_pk + a.b_pk_n);

    int oa[NA], ob[NB];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int e = lane + q * kWave;
        oa[q] = (e < M * K) ? (e / K) * LDK + (e % K) : -1;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = lane + q * kWave;
        ob[q] = (e < K * N) ? (e % N) * LDK + (e / N) : -1;
    }
    const int r32 = lane & 31, h = lane >> 5;

    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;

    const int64_t p0 = a.seg[c - a.c0], p_end = a.seg[c - a.c0 + 1];
    uint32_t pa[NA], pb[NB];
    unsigned short la[T == 3 ? NA : 1], lb[T == 3 ? NB : 1];
    auto prefetch = [&](int64_t p) {
        const int64_t oa0 = a.a_blk_off[a.stk_a[p]], ob0 = a.b_blk_off[a.stk_b[p]];
        const uint32_t *ga = a.a_pk + oa0;
        const uint32_t *gb = a.b_pk + ob0;
#pragma unroll
        for (int q = 0; q < NA; ++q) pa[q] = (oa[q] >= 0) ? ga[lane + q * kWave] : 0u;
#pragma unroll
        for (int q = 0; q < NB; ++q) pb[q] = (ob[q] >= 0) ? gb[lane + q * kWave] : 0u;
        if (T == 3) {
#pragma unroll
            for (int q = 0; q < NA; ++q) la[q] = (oa[q] >= 0) ? alo3[oa0 + lane + q * kWave] : 0;
#pragma unroll
            for (int q = 0; q < NB; ++q) lb[q] = (ob[q] >= 0) ? blo3[ob0 + lane + q * kWave] : 0;
        }
    };
    if (p0 < p_end) prefetch(p0);
    __syncthreads();
    for (int64_t p = p0; p < p_end; ++p) {
#pragma unroll
        for (int q = 0; q < NA; ++q)
            if (oa[q] >= 0) {
                as[oa[q]] = static_cast<unsigned short>(pa[q] >> 16);
                as[PLANE + oa[q]] = static_cast<unsigned short>(pa[q] & 0xFFFFu);
                if (T == 3) as[2 * PLANE + oa[q]] = la[q];
            }
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (ob[q] >= 0) {
                bs[ob[q]] = static_cast<unsigned short>(pb[q] >> 16);
                bs[PLANE + ob[q]] = static_cast<unsigned short>(pb[q] & 0xFFFFu);
                if (T == 3) bs[2 * PLANE + ob[q]] = lb[q];
            }
        __syncthreads();
        if (p + 1 < p_end) prefetch(p + 1);
        bf16_split_product<T, KS, LDK, PLANE>(as, bs, r32 * LDK + 8 * h, acc);
        __syncthreads();
    }
    lp_store<M, N>(a, c, acc, [&](int q, int &row, int &col) {
        row = 8 * (q >> 2) + 4 * h + (q & 3);
        col = r32;
    });
}

// ------------------------------------------------------------------ FP32
// One wavefront per C block as a 2 x 2 grid of 16 x 16 tiles.
// Lane layout of V_MFMA_F32_16X16X4_F32 (measured on gfx950):
// A(i,k): lane i + 16k; B(k,j): lane j + 16k; D(i,j): lane j + 16*(i/4),
// register i%4.
template <int M, int N, int K>
__global__ void __launch_bounds__(64)
k_smm_f32(SmmArgs a) {
    constexpr int LDA = 33, LDB = 32;               // A rows in distinct banks
    constexpr int KP = 4 * ((K + 3) / 4);
    constexpr int MT = (M + 15) / 16, NT = (N + 15) / 16;
    constexpr int NA = (M * K + kWave - 1) / kWave, NB = (K * N + kWave - 1) / kWave;
    __shared__ float sA[32 * LDA];
    __shared__ float sB[KP * LDB];
    const int64_t item = lp_item(a.nC);
    if (item >= a.nC) return;
    const int lane = threadIdx.x;
    const int64_t c = a.worklist ? a.worklist[a.c0 + item] : a.c0 + item;
    for (int e = lane; e < 32 * LDA; e += kWave) sA[e] = 0.f;
    for (int e = lane; e < KP * LDB; e += kWave) sB[e] = 0.f;
    int oa[NA], ob[NB];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int e = lane + q * kWave;
        oa[q] = (e < M * K) ? (e / K) * LDA + (e % K) : -1;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = lane + q * kWave;
        ob[q] = (e < K * N) ? (e / N) * LDB + (e % N) : -1;
    }
    const int r16 = lane & 15, kq = lane >> 4;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;

    const int64_t p0 = a.seg[c - a.c0], p_end = a.seg[c - a.c0 + 1];
    uint32_t pa[NA], pb[NB];
    auto prefetch = [&](int64_t p) {
        const uint32_t *ga = a.a_pk + a.a_blk_off[a.stk_a[p]];
        const uint32_t *gb = a.b_pk + a.b_blk_off[a.stk_b[p]];
#pragma unroll
        for (int q = 0; q < NA; ++q) pa[q] = (oa[q] >= 0) ? ga[lane + q * kWave] : 0u;
#pragma unroll
        for (int q = 0; q < NB; ++q) pb[q] = (ob[q] >= 0) ? gb[lane + q * kWave] : 0u;
    };
    if (p0 < p_end) prefetch(p0);
    __syncthreads();
    for (int64_t p = p0; p < p_end; ++p) {
#pragma unroll
        for (int q = 0; q < NA; ++q)
            if (oa[q] >= 0) sA[oa[q]] = __uint_as_float(pa[q]);
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (ob[q] >= 0) sB[ob[q]] = __uint_as_float(pb[q]);
        __syncthreads();
        if (p + 1 < p_end) prefetch(p + 1);
        f4 part[2][2] = {};
#pragma unroll
        for (int ks = 0; ks < KP / 4; ++ks) {
            float av[2], bv[2];
#pragma unroll
            for (int t = 0; t < MT; ++t) av[t] = sA[(16 * t + r16) * LDA + 4 * ks + kq];
#pragma unroll
            for (int u = 0; u < NT; ++u) bv[u] = sB[(4 * ks + kq) * LDB + 16 * u + r16];
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    part[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], bv[u], part[t][u],
                                                                      0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[(t * 2 + u) * 4 + r] += static_cast<double>(part[t][u][r]);
        __syncthreads();
    }
    lp_store<M, N>(a, c, acc, [&](int q, int &row, int &col) {
        const int tile = q >> 2, r = q & 3;
        const int t = tile >> 1, u = tile & 1;
        row = 16 * t + 4 * kq + r;
        col = 16 * u + r16;
        if (t >= MT || u >= NT) row = 1 << 20;   // tile not present
    });
}

// ------------------------------------------------------------------ quads
// The quad scheme of the FP64 path (smm_quad.hip) with the reduced-precision
// products above: four waves per 2 x 2 quad of C blocks; per entry k wave w
// stages operand w (A(i_0, k), A(i_1, k), B(k, j_0), B(k, j_1); each read
// from HBM once) into its LDS slot in the layout the MFMA reads need, and
// computes C block (w / 2, w % 2) when the entry holds that product.  Each
// block product is accumulated in FP32 and added into the FP64 sum of its C
// block, in ascending k, exactly as in the one-block-per-wave kernels.
__device__ inline int4 lp_uniform4(int4 v) {
    return make_int4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                     __builtin_amdgcn_readfirstlane(v.z), __builtin_amdgcn_readfirstlane(v.w));
}

// T = 0: FP32; T = 2 or 3: split-BF16 with that many parts.  Occupancy
// target: five waves per SIMD for two parts (96 registers, no spills; 5%
// faster per sign than four on the 2048-site workload at eps 1e-5; six
// spill and are slower), four otherwise (three parts need 124 registers).
template <int S, int T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(T == 2 ? 5 : 4, 8)))
k_lowp_quad(SmmArgs a) {
    constexpr bool BF = T >= 2;
    constexpr int NP = BF ? T : 1;                      // bf16 planes per operand
    constexpr int B2 = S * S;
    constexpr int NV = (B2 + kWave - 1) / kWave;
    constexpr int LDK = 40, PLANE = 32 * LDK;           // split-BF16: [32][LDK] planes
    constexpr int LDA = 33, LDB = 32, KP = 4 * ((S + 3) / 4);
    constexpr int FA = 32 * LDA, FB = KP * LDB;          // FP32: A [32][LDA], B [KP][LDB]
    constexpr int BYTES = BF ? 4 * NP * PLANE * 2 : (2 * FA + 2 * FB) * 4;
    __shared__ __attribute__((aligned(16))) unsigned char smem[BYTES];
    __shared__ int4 ebuf[2][64];
    unsigned short *us = reinterpret_cast<unsigned short *>(smem);
    float *fs = reinterpret_cast<float *>(smem);

    const int64_t per = (a.n_quads + kXcds - 1) / kXcds;
    const int64_t it = static_cast<int64_t>(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    if (it >= a.n_quads) return;
    const int64_t item = a.q_order ? a.q_order[it] : it;
    const int lane = threadIdx.x % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
    const int rr = wv >> 1, cc = wv & 1;                // this wave's C block (rr, cc)

    for (int e = threadIdx.x; e < BYTES / 4; e += 256) reinterpret_cast<uint32_t *>(smem)[e] = 0u;
    // LDS position of element lane + 64 v of this wave's operand (-1: none),
    // recomputed where it is used (fewer live registers)
    auto lds_off = [&](int v) {
        const int e = lane + v * kWave;
        int o = -1;
        if (e < B2) {
            const int i = e / S, j = e % S;            // row, column of the stored block
            if (BF) o = (wv < 2) ? i * LDK + j : j * LDK + i;
            else o = (wv < 2) ? wv * FA + i * LDA + j : 2 * FA + (wv - 2) * FB + i * LDB + j;
        }
        return o;
    };

    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;

    constexpr int kEntryChunk = 64;
    const int64_t e0 = a.q_seg[item], ne = a.q_seg[item + 1] - e0;
    const int4 none = make_int4(-1, -1, -1, -1);
    auto pick = [](const int4 v, int z) { return z == 0 ? v.x : z == 1 ? v.y : z == 2 ? v.z : v.w; };
    uint32_t pv[NV];
    unsigned short pl[T == 3 ? NV : 1];
    const unsigned short *lo3 = reinterpret_cast<const unsigned short *>(
        wv < 2 ? a.a_pk + a.a_pk_n : a.b_pk + a.b_pk_n);
    auto load_block = [&](const int4 en) {
        const int id = pick(en, wv);
        if (id >= 0) {
            const int64_t o0 = static_cast<int64_t>(id) * B2;
            const uint32_t *g = (wv < 2 ? a.a_pk : a.b_pk) + o0;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < NV - 1 || lane + v * kWave < B2) pv[v] = g[lane + v * kWave];
            if (T == 3) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v < NV - 1 || lane + v * kWave < B2) pl[v] = lo3[o0 + lane + v * kWave];
            }
        }
    };
    int4 creg = none;
    if (wv == 0) {
        if (lane < ne) ebuf[0][lane] = a.q_ent[e0 + lane];
        if (kEntryChunk + lane < ne) creg = a.q_ent[e0 + kEntryChunk + lane];
    }
    __syncthreads();
    int4 nxt = none;
    if (ne > 0) {
        nxt = lp_uniform4(ebuf[0][0]);
        load_block(nxt);
    }
    const int r32 = lane & 31, h = lane >> 5, r16 = lane & 15, kq = lane >> 4;
    for (int64_t t = 0; t < ne; ++t) {
        const int4 cur = nxt;
        if (pick(cur, wv) >= 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (const int o = lds_off(v); o >= 0) {
                    if (BF) {
                        const int plane = NP * wv;
                        us[plane * PLANE + o] = static_cast<unsigned short>(pv[v] >> 16);
                        us[(plane + 1) * PLANE + o] = static_cast<unsigned short>(pv[v] & 0xFFFFu);
                        if (T == 3) us[(plane + 2) * PLANE + o] = pl[v];
                    } else {
                        fs[o] = __uint_as_float(pv[v]);
                    }
                }
        }
        const int64_t t1 = t + 1;
        if ((t1 % kEntryChunk) == 0 && t1 < ne && wv == 0) {
            ebuf[(t1 / kEntryChunk) & 1][lane] = creg;
            if (t1 + kEntryChunk + lane < ne) creg = a.q_ent[e0 + t1 + kEntryChunk + lane];
        }
        __syncthreads();
        if (t1 < ne) {
            nxt = lp_uniform4(ebuf[(t1 / kEntryChunk) & 1][t1 % kEntryChunk]);
            load_block(nxt);
        }
        if (pick(cur, rr) >= 0 && pick(cur, 2 + cc) >= 0) {
            if (BF) {
                const unsigned short *as = us + (NP * rr) * PLANE;
                const unsigned short *bs = us + (NP * (2 + cc)) * PLANE;
                constexpr int KS = (S + 15) / 16;
                bf16_split_product<BF ? T : 2, KS, LDK, PLANE>(as, bs, r32 * LDK + 8 * h, acc);
            } else {
                const float *sA = fs + rr * FA, *sB = fs + 2 * FA + cc * FB;
                constexpr int MT = (S + 15) / 16;
                f4 part[2][2] = {};
#pragma unroll
                for (int ks = 0; ks < KP / 4; ++ks) {
                    float av[2], bv[2];
#pragma unroll
                    for (int tt = 0; tt < MT; ++tt) av[tt] = sA[(16 * tt + r16) * LDA + 4 * ks + kq];
#pragma unroll
                    for (int u = 0; u < MT; ++u) bv[u] = sB[(4 * ks + kq) * LDB + 16 * u + r16];
#pragma unroll
                    for (int tt = 0; tt < MT; ++tt)
#pragma unroll
                        for (int u = 0; u < MT; ++u)
                            part[tt][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[tt], bv[u],
                                                                              part[tt][u], 0, 0, 0);
                }
#pragma unroll
                for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[(tt * 2 + u) * 4 + q] += static_cast<double>(part[tt][u][q]);
            }
        }
        __syncthreads();
    }

    // epilogue: this wave's C block
    const int64_t cb = a.q_cblk[4 * item + 2 * rr + cc];
    if (cb < 0) return;
    const int64_t co = a.c_blk_off[cb];
    const double *cin = nullptr;
    if (a.cin_map) {
        const int64_t tt = a.cin_map[cb];
        if (tt >= 0) cin = a.cin_vals + a.cin_blk_off[tt];
    }
    double sq = 0.0, mx = 0.0;
    constexpr int MT = (S + 15) / 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        int row, col;
        if (BF) {
            row = 8 * (q >> 2) + 4 * h + (q & 3);
            col = r32;
        } else {
            const int tile = q >> 2, tt = tile >> 1, u = tile & 1;
            row = 16 * tt + 4 * kq + (q & 3);
            col = 16 * u + r16;
            if (tt >= MT || u >= MT) row = 1 << 20;
        }
        if (row < S && col < S) {
            double v = a.alpha * acc[q];
            if (cin) v += a.beta * cin[row * S + col];
            a.c_vals[co + row * S + col] = v;
            sq += v * v;
            mx = fmax(mx, fabs(v));
        }
    }
    sq = lp_wave_sum(sq);
    mx = lp_wave_max(mx);
    if (lane == 0) {
        a.sq_out[cb] = sq;
        a.mx_out[cb] = mx;
        if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
    }
}

int launch_lowp_quad(const SmmArgs &a, hipStream_t s) {
    if (a.n_quads <= 0) return BSM_OK;
    const int64_t per = (a.n_quads + kXcds - 1) / kXcds;
    const int64_t grid = per * kXcds;
    if (grid > (1ll << 31) - 1) { set_error("too many quads in one launch"); return BSM_EINVAL; }
    const unsigned g = static_cast<unsigned>(grid);
#define BSM_LQ(SZ)                                                            \
    case SZ:                                                                  \
        if (a.prec == BSM_SPLIT_BF16) BSM_LAUNCH((k_lowp_quad<SZ, 2>), g, 256, 0, s)(a);\
        else if (a.prec == BSM_SPLIT_BF16X3) BSM_LAUNCH((k_lowp_quad<SZ, 3>), g, 256, 0, s)(a); \
        else BSM_LAUNCH((k_lowp_quad<SZ, 0>), g, 256, 0, s)(a);                         \
        break;
    switch (a.uni_m) {
        BSM_LQ(5)
        BSM_LQ(13)
        BSM_LQ(23)
        BSM_LQ(26)
        BSM_LQ(32)
        default: set_error("no reduced-precision quad kernel for block size %d", a.uni_m); return BSM_EINVAL;
    }
#undef BSM_LQ
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bool smm_lowp_available(int m, int n, int k) {
    return (m == n && n == k) && (m == 5 || m == 13 || m == 23 || m == 26 || m == 32);
}

int smm_launch_lowp(const SmmArgs &a, hipStream_t s) {
    if (a.nC <= 0) return BSM_OK;
    const int64_t per = (a.nC + kXcds - 1) / kXcds;
    const unsigned grid = static_cast<unsigned>(per * kXcds);
    if (!(a.uni_m && smm_lowp_available(a.uni_m, a.uni_n, a.uni_k))) {
        set_error("reduced-precision products need uniform block sizes 5, 13, 23, 26 or 32");
        return BSM_EINVAL;
    }
#define BSM_LP(SZ)                                                                  \
    case SZ:                                                                        \
        if (a.prec == BSM_FP32) BSM_LAUNCH((k_smm_f32<SZ, SZ, SZ>), grid, 64, 0, s)(a);       \
        else if (a.prec == BSM_SPLIT_BF16X3) BSM_LAUNCH((k_smm_bf16x3<SZ, SZ, SZ, 3>), grid, 64, 0, s)(a); \
        else BSM_LAUNCH((k_smm_bf16x3<SZ, SZ, SZ, 2>), grid, 64, 0, s)(a);                    \
        break;
    switch (a.uni_m) {
        BSM_LP(5)
        BSM_LP(13)
        BSM_LP(23)
        BSM_LP(26)
        BSM_LP(32)
        default: break;
    }
#undef BSM_LP
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
