// FP64 block products for mixed block sizes in {5, 13, 23, 26}: every
// (m, n) class of a chunk in one persistent launch, with the operand sharing
// of the uniform quad kernel (smm_quad.hip).
//
// The work items are 2 x 2 groups of C blocks over paired rows and paired
// columns of equal size (quad.hip, MAP), so all four C blocks of an item are
// m x n and only k changes from entry to entry.  A fixed grid of four-wave
// workgroups takes items from an atomic counter until none is left; each
// item dispatches once on its (m, n) class to compile-time code, and each
// entry on its k.  Per entry wave w stages operand w (A(i_0, k), A(i_1, k),
// B(k, j_0), B(k, j_1)), each read from HBM once, into its LDS slot exactly
// as it sits in HBM, and then multiplies C block (w / 2, w % 2) when the
// entry holds that product.  The products and their order are those of the
// per-class kernel (k_smm_f64_class: the same V_MFMA_F64_4X4X4_4B_F64
// sequence per product, ascending k per C block), so the results are the
// same bits.
//
// Entry metadata (operand offsets and k) is read for 64 entries at a time by
// wave 0, one entry per lane, and kept in LDS: the entries of chunk c + 2 are
// loaded at the start of chunk c, their operand offsets (which depend on
// them) at the start of chunk c + 1, so no load of an iteration waits on
// another load of the same iteration.
#include <cstdlib>

#include "smm.h"

namespace bsm {

namespace {

constexpr int kMqSlot = 26 * 26;                    // LDS doubles of one operand slot
constexpr int kMqTail = 4 * 26 + 8 * 26 + 8;        // padded reads past the last slot
constexpr int kMqChunk = 64;
constexpr int kMqWaves = 4;
constexpr int kMqNV = (kMqSlot + kWave - 1) / kWave;  // operand doubles per lane

__device__ inline double mq_wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double mq_wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
// The class bodies are out-of-line calls.  Handed the kernel's SmmArgs by a
// plain reference, the compiler copies the struct to the stack and reaches
// every field, and through the fields every operand, with flat (generic)
// instructions; a reference into the kernel-argument segment (address space
// 4) and global-space views of the data pointers give global loads and
// stores instead (10% less time on the mixed workload, same code otherwise).
using KArgs = const __attribute__((address_space(4))) SmmArgs;
template <class T>
__device__ inline const T *gcp(const T *p) {
    return (const T *)(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ inline T *gp(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)p;
}
// The same, read once for the wave (scalar registers).
template <class T>
__device__ inline const T *ugcp(const T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v)));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32)));
    return (const T *)(const __attribute__((address_space(1))) T *)((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ inline int64_t mq_uniform64(int64_t v) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v)));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32)));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// One product A (M x K, at sA) times B (K x N, at sB), both row-major in LDS,
// into the lane's accumulators; the instruction sequence of the per-class
// kernel's compile-time-k step.
template <int M, int N, int K, int HR, int HC>
__device__ inline void mq_compute(const double *sA, const double *sB, int bh, int bw, int x, int y,
                                  double (&acc)[HR][HC]) {
    constexpr int KS = (K + 3) / 4, KLAST = K - 4 * (KS - 1);
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

struct MqMeta {
    int64_t off[2][kMqChunk][4];   // operand offsets of an entry (-1: absent)
    int32_t k[2][kMqChunk];        // k of an entry
};

// Wave 0: operand offsets and k of the entry en (M rows in the A blocks).
template <int M>
__device__ inline void mq_offsets(const int64_t *abo, const int64_t *bbo, int4 en,
                                  int64_t (&o)[4], int32_t &kk) {
    o[0] = en.x >= 0 ? abo[en.x] : -1;
    o[1] = en.y >= 0 ? abo[en.y] : -1;
    o[2] = en.z >= 0 ? bbo[en.z] : -1;
    o[3] = en.w >= 0 ? bbo[en.w] : -1;
    const int ai = en.x >= 0 ? en.x : en.y;
    kk = ai >= 0 ? static_cast<int32_t>((abo[ai + 1] - abo[ai]) / M) : 0;
}

// One work item (group) of class (M, N); EPS entries are staged per barrier
// pair (slot set q of LDS holds entry t + q).
template <int M, int N, int EPS>
__device__ inline void mq_item(KArgs &a, int64_t item, double *sm, MqMeta &md) {
    constexpr int MT = (M + 3) / 4, NT = (N + 3) / 4;
    constexpr int HR = (MT + 1) / 2, HC = (NT + 1) / 2;
    const int lane = threadIdx.x % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
    const int rr = wv >> 1, cc = wv & 1;
    const int x = lane >> 4, blk = (lane >> 2) & 3, y = lane & 3;
    const int bh = blk >> 1, bw = blk & 1;
    const auto qseg = ugcp(a.q_seg);
    const auto qent = ugcp(a.q_ent);
    const auto abo = ugcp(a.a_blk_off), bbo = ugcp(a.b_blk_off);
    const auto avals = ugcp(a.a_vals), bvals = ugcp(a.b_vals);
    const int64_t e0 = qseg[item], ne = qseg[item + 1] - e0;

    double acc[HR][HC];
#pragma unroll
    for (int t = 0; t < HR; ++t)
#pragma unroll
        for (int u = 0; u < HC; ++u) acc[t][u] = 0.0;

    // metadata pipeline (wave 0): chunk 0 into LDS now, chunk 1's offsets
    // and chunk 2's entries into registers
    int64_t roff[4] = {-1, -1, -1, -1};
    int32_t rk = 0;
    int4 creg = make_int4(-1, -1, -1, -1);
    if (wv == 0) {
        if (lane < ne) {
            int64_t o[4];
            int32_t kk;
            mq_offsets<M>(abo, bbo, qent[e0 + lane], o, kk);
#pragma unroll
            for (int z = 0; z < 4; ++z) md.off[0][lane][z] = o[z];
            md.k[0][lane] = kk;
        }
        if (kMqChunk + lane < ne) mq_offsets<M>(abo, bbo, qent[e0 + kMqChunk + lane], roff, rk);
        if (2 * kMqChunk + lane < ne) creg = qent[e0 + 2 * kMqChunk + lane];
    }
    __syncthreads();

    // entry t's metadata from LDS (wave-uniform): present operands, this
    // wave's operand offset, k
    auto fetch = [&](int64_t t, unsigned &hm, int64_t &my_off, int &kk) {
        hm = 0;
        my_off = -1;
        kk = 0;
        if (t >= ne) return;
        const int b = static_cast<int>((t / kMqChunk) & 1), i = static_cast<int>(t % kMqChunk);
#pragma unroll
        for (int z = 0; z < 4; ++z) {
            const int64_t o = mq_uniform64(md.off[b][i][z]);
            if (o >= 0) hm |= 1u << z;
            if (z == wv) my_off = o;
        }
        kk = __builtin_amdgcn_readfirstlane(md.k[b][i]);
    };
    double pv[EPS][kMqNV];
    auto load_op = [&](int64_t off, int kk, double (&p)[kMqNV]) {
        if (off < 0) return;
        const auto g = (wv < 2 ? avals : bvals) + off;
        const int len = (wv < 2 ? M : N) * kk;
#pragma unroll
        for (int v = 0; v < kMqNV; ++v)
            if (lane + v * kWave < len) p[v] = g[lane + v * kWave];
    };

    unsigned nhm[EPS];
    int64_t noff[EPS];
    int nk[EPS];
#pragma unroll
    for (int q = 0; q < EPS; ++q) {
        fetch(q, nhm[q], noff[q], nk[q]);
        load_op(noff[q], nk[q], pv[q]);
    }
    for (int64_t t = 0; t < ne; t += EPS) {
        unsigned hm[EPS];
        int k[EPS];
#pragma unroll
        for (int q = 0; q < EPS; ++q) {
            hm[q] = nhm[q];
            k[q] = nk[q];
            if ((hm[q] >> wv) & 1u) {
                const int len = (wv < 2 ? M : N) * k[q];
                double *slot = sm + (4 * q + wv) * kMqSlot;
#pragma unroll
                for (int v = 0; v < kMqNV; ++v)
                    if (lane + v * kWave < len) slot[lane + v * kWave] = pv[q][v];
            }
        }
        const int64_t t1 = t + EPS;
        if ((t1 % kMqChunk) == 0 && t1 < ne && wv == 0) {
            // entering chunk t1 / 64: its metadata (ready in registers) goes
            // to LDS; the next chunk's offsets and the one after's entries
            // are loaded
            const int b = static_cast<int>((t1 / kMqChunk) & 1);
#pragma unroll
            for (int z = 0; z < 4; ++z) md.off[b][lane][z] = roff[z];
            md.k[b][lane] = rk;
            if (t1 + kMqChunk + lane < ne) mq_offsets<M>(abo, bbo, creg, roff, rk);
            if (t1 + 2 * kMqChunk + lane < ne) creg = qent[e0 + t1 + 2 * kMqChunk + lane];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPS; ++q) {
            fetch(t1 + q, nhm[q], noff[q], nk[q]);
            load_op(noff[q], nk[q], pv[q]);
        }
#pragma unroll
        for (int q = 0; q < EPS; ++q) {
            if (((hm[q] >> rr) & 1u) && ((hm[q] >> (2 + cc)) & 1u)) {
                const double *sA = sm + (4 * q + rr) * kMqSlot, *sB = sm + (4 * q + 2 + cc) * kMqSlot;
                switch (k[q]) {
                    case 5: mq_compute<M, N, 5, HR, HC>(sA, sB, bh, bw, x, y, acc); break;
                    case 13: mq_compute<M, N, 13, HR, HC>(sA, sB, bh, bw, x, y, acc); break;
                    case 23: mq_compute<M, N, 23, HR, HC>(sA, sB, bh, bw, x, y, acc); break;
                    case 26: mq_compute<M, N, 26, HR, HC>(sA, sB, bh, bw, x, y, acc); break;
                    default: break;
                }
            }
        }
        __syncthreads();
    }

    // epilogue: this wave's C block
    const int64_t cb = gcp(a.q_cblk)[4 * item + 2 * rr + cc];
    if (cb >= 0) {
        const int64_t co = gcp(a.c_blk_off)[cb];
        const double *cin = nullptr;
        if (a.cin_map) {
            const int64_t tt = gcp(a.cin_map)[cb];
            if (tt >= 0) cin = gcp(a.cin_vals) + gcp(a.cin_blk_off)[tt];
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
                    gp(a.c_vals)[co + row * N + col] = v;
                    sq += v * v;
                    mx = fmax(mx, fabs(v));
                }
            }
        sq = mq_wave_sum(sq);
        mx = mq_wave_max(mx);
        if (lane == 0) {
            gp(a.sq_out)[cb] = sq;
            gp(a.mx_out)[cb] = mx;
            if (!isfinite(sq)) atomicOr(a.flags, kFlagNonFinite);
        }
    }
}

// Class of item (m, n) from its first C block: 4 class(m) + class(n), or -1.
template <class A>
__device__ inline int mq_class(A &a, int64_t item) {
    int64_t cb = -1;
    for (int z = 0; z < 4 && cb < 0; ++z) cb = a.q_cblk[4 * item + z];
    if (cb < 0) return -1;
    auto cls = [](int b) { return b == 5 ? 0 : b == 13 ? 1 : b == 23 ? 2 : b == 26 ? 3 : -1; };
    const int cm = cls(a.c_rbs[a.c_row[cb]]), cn = cls(a.c_cbs[a.c_col[cb]]);
    return (cm < 0 || cn < 0) ? -1 : 4 * cm + cn;
}

// The next work item from the counter into s_item, its class into s_cls
// (-1 past the end); every wave of the workgroup sees both.
__device__ inline void mq_next(KArgs &a, int64_t n_items, unsigned long long *counter,
                               int64_t &s_item, int &s_cls, int64_t &it, int &cls) {
    if (threadIdx.x == 0) {
        const int64_t x = static_cast<int64_t>(atomicAdd(counter, 1ull));
        s_item = x;
        s_cls = x < n_items ? mq_class(a, a.q_order ? a.q_order[x] : x) : -1;
    }
    __syncthreads();
    it = s_item;
    cls = s_cls;
    __syncthreads();                 // s_item, s_cls are rewritten by the next call
}

// Items of class (M, N) from `it` on, taking the next item from the counter
// until one of another class (or none) comes: the work order lists a
// class's groups together, so a workgroup enters this once per class it
// meets rather than once per group.  Returns that item; *cls its class.
template <int M, int N, int EPS>
__device__ __attribute__((noinline)) int64_t
mq_run(KArgs &a, int64_t n_items, unsigned long long *counter, int64_t it, int *cls,
       double *sm, MqMeta &md, int64_t &s_item, int &s_cls) {
    const int me = *cls;
    int c = me;
    while (it < n_items && c == me) {
        mq_item<M, N, EPS>(a, a.q_order ? a.q_order[it] : it, sm, md);
        mq_next(a, n_items, counter, s_item, s_cls, it, c);
    }
    *cls = c;
    return it;
}

// EPS entries per barrier pair; WPE: the occupancy target (LDS allows five
// workgroups per CU with one entry per stage, three with two).
template <int EPS, int WPE>
__global__ void __launch_bounds__(64 * kMqWaves) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_smm_f64_mquad(SmmArgs a, unsigned long long *counter) {
    static_assert(kMqChunk % EPS == 0, "stages must not straddle metadata chunks");
    __shared__ double sm[EPS * 4 * kMqSlot + kMqTail];
    __shared__ MqMeta md;
    __shared__ int64_t s_item;
    __shared__ int s_cls;
    for (int e = EPS * 4 * kMqSlot + static_cast<int>(threadIdx.x); e < EPS * 4 * kMqSlot + kMqTail;
         e += 64 * kMqWaves)
        sm[e] = 0.0;
    const int64_t n_items = a.n_quads_dev ? *a.n_quads_dev : a.n_quads;
    // a is the first explicit argument: offset 0 of the kernel-argument segment
    KArgs &ka = *(KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    int64_t it = 0;
    int cls = -1;
    mq_next(ka, n_items, counter, s_item, s_cls, it, cls);
    while (it < n_items) {           // it and cls are the same in every wave
        switch (cls) {
#define BSM_MQ(ID, MM, NN) \
    case ID: it = mq_run<MM, NN, EPS>(ka, n_items, counter, it, &cls, sm, md, s_item, s_cls); break;
            BSM_MQ(0, 5, 5) BSM_MQ(1, 5, 13) BSM_MQ(2, 5, 23) BSM_MQ(3, 5, 26)
            BSM_MQ(4, 13, 5) BSM_MQ(5, 13, 13) BSM_MQ(6, 13, 23) BSM_MQ(7, 13, 26)
            BSM_MQ(8, 23, 5) BSM_MQ(9, 23, 13) BSM_MQ(10, 23, 23) BSM_MQ(11, 23, 26)
            BSM_MQ(12, 26, 5) BSM_MQ(13, 26, 13) BSM_MQ(14, 26, 23) BSM_MQ(15, 26, 26)
#undef BSM_MQ
            default: mq_next(ka, n_items, counter, s_item, s_cls, it, cls); break;
        }
    }
}

__global__ void k_mq_zero(unsigned long long *p) { *p = 0ull; }

// Work order of the groups: by class, the classes with the most work per
// product first (m n descending), ascending group index inside a class, so
// that the workgroups of a CU run the same class's code at the same time
// (the sixteen class bodies together exceed the instruction cache) and a
// class's groups keep their spatial order.
constexpr int kMqOrderThreads = 1024;
__device__ inline int mq_rank_of_class(int cls) {
    // class 4 cm + cn of sizes {5, 13, 23, 26}, ranked by m n descending
    // (676, 598, 598, 529, 338, 338, 299, 299, 169, 130, 130, 115, 115, 65, 65, 25)
    constexpr int rank[16] = {15, 13, 11, 9, 14, 8, 6, 4, 12, 7, 3, 1, 10, 5, 2, 0};
    return cls < 0 ? 15 : rank[cls];
}

// Groups counted in device memory (a.n_quads_dev) or a.n_quads.
__device__ inline int64_t mq_count(const SmmArgs &a) {
    return a.n_quads_dev ? *a.n_quads_dev : a.n_quads;
}

__global__ void k_mq_class_of(SmmArgs a, int8_t *rank) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= mq_count(a)) return;
    rank[q] = static_cast<int8_t>(mq_rank_of_class(mq_class(a, q)));
}

// One workgroup per rank r: the positions of rank r's groups, in ascending
// group order, after every group of a smaller rank.
__global__ void __launch_bounds__(kMqOrderThreads)
k_mq_order(const int8_t *rank, SmmArgs a, int64_t *order) {
    const int64_t n = mq_count(a);
    __shared__ int64_t s_wave[kMqOrderThreads / kWave];
    __shared__ int64_t s_base, s_run;
    const int r = blockIdx.x;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    // groups of smaller rank
    int64_t before = 0;
    for (int64_t q = threadIdx.x; q < n; q += kMqOrderThreads) before += rank[q] < r ? 1 : 0;
    for (int o = kWave / 2; o > 0; o >>= 1) before += __shfl_xor(before, o, kWave);
    if (lane == 0) s_wave[wid] = before;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t b = 0;
        for (int w = 0; w < kMqOrderThreads / kWave; ++w) b += s_wave[w];
        s_base = b;
        s_run = 0;
    }
    __syncthreads();
    for (int64_t q0 = 0; q0 < n; q0 += kMqOrderThreads) {
        const int64_t q = q0 + threadIdx.x;
        const int mine = (q < n && rank[q] == r) ? 1 : 0;
        // block-wide exclusive scan of `mine`
        const unsigned long long ball = __ballot(mine);
        const int in_wave = __popcll(ball & ((1ull << lane) - 1ull));
        __syncthreads();
        if (lane == 0) s_wave[wid] = __popcll(ball);
        __syncthreads();
        int64_t off = 0;
        for (int w = 0; w < wid; ++w) off += s_wave[w];
        if (mine) order[s_base + s_run + off + in_wave] = q;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int w = 0; w < kMqOrderThreads / kWave; ++w) t += s_wave[w];
            s_run += t;
        }
    }
}

}  // namespace

int mquad_order(const SmmArgs &a, int8_t *rank_scratch, int64_t *order, hipStream_t s) {
    if (a.n_quads <= 0) return BSM_OK;
    k_mq_class_of<<<grid_for(a.n_quads, 256), 256, 0, s>>>(a, rank_scratch);
    k_mq_order<<<16, kMqOrderThreads, 0, s>>>(rank_scratch, a, order);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// Entries staged per barrier pair (1 or 2); BSM_MQUAD_STAGE overrides the
// default.  Two halve the barriers per entry but take occupancy from four
// workgroups per CU to three: 9.6 s per sign on the mixed workload against
// 8.3 s with one.
static int mquad_stage() {
    const char *e = getenv("BSM_MQUAD_STAGE");
    return (e && atoi(e) == 2) ? 2 : 1;
}

int launch_mquad(const SmmArgs &a, hipStream_t s) {
    if (a.n_quads <= 0) return BSM_OK;
    if (!a.counter) { set_error("internal: mixed quads need a work counter"); return BSM_EINVAL; }
    int dev = 0, cus = 256;
    BSM_HIP(hipGetDevice(&dev));
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // workgroups resident per CU: LDS (about 29 KB each with one entry per
    // stage, 50 KB with two) allows five or three
    const int eps = mquad_stage();
    const int64_t want = static_cast<int64_t>(cus) * (eps == 2 ? 3 : 5);
    const unsigned grid = static_cast<unsigned>(want < a.n_quads ? want : a.n_quads);
    k_mq_zero<<<1, 1, 0, s>>>(a.counter);
    if (eps == 2) BSM_LAUNCH((k_smm_f64_mquad<2, 3>), grid, 64 * kMqWaves, 0, s)(a, a.counter);
    else BSM_LAUNCH((k_smm_f64_mquad<1, 4>), grid, 64 * kMqWaves, 0, s)(a, a.counter);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
