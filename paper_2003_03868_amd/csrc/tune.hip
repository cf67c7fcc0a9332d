// Autotuning support: the per-(m, n, k) kernel-parameter table the multiply
// consults, and a benchmark that times parameter sets on a synthetic product
// stack of one (m, n, k) (the paper's autotuner explores kernel parameters per
// (m, n, k) on batches of products, "Batched execution" subsection).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "smm.h"

namespace bsm {

namespace {
std::mutex g_tab_mu;
std::map<std::tuple<int, int, int>, SmmParams> g_tab;

// SplitMix64 finaliser: a counter-based generator for synthetic data.
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
}  // namespace

bool table_lookup(int m, int n, int k, SmmParams *out) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tab.find({m, n, k});
    if (it == g_tab.end()) return false;
    *out = it->second;
    return true;
}

void table_set(int count, const int32_t *mnk, const SmmParams *prm) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    if (count < 0) { g_tab.clear(); return; }
    for (int i = 0; i < count; ++i) g_tab[{mnk[3 * i], mnk[3 * i + 1], mnk[3 * i + 2]}] = prm[i];
}

__global__ void k_bench_fill(double *v, int64_t n, uint64_t seed) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] = static_cast<double>(mix64(seed ^ static_cast<uint64_t>(i)) >> 11) * 0x1.0p-53 - 0.5;
}

// Product p of C block c: A block and B block drawn from pools of `pool`
// blocks per k value; every product of one C block uses the same k slot
// rotation so that consecutive products visit all k values of the set.
__global__ void k_bench_stack(int64_t nprod, int per_c, int pool, int nk, uint64_t seed,
                              int32_t *stk_a, int32_t *stk_b) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= nprod) return;
    const int64_t c = p / per_c, i = p % per_c;
    const int slot = static_cast<int>((c + i) % nk);
    const uint64_t h = mix64(seed ^ (static_cast<uint64_t>(p) * 0x632BE59BD9B4E019ull));
    stk_a[p] = slot * pool + static_cast<int32_t>(h % pool);
    stk_b[p] = slot * pool + static_cast<int32_t>((h >> 32) % pool);
}

__global__ void k_bench_iota(int64_t *v, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

__global__ void k_bench_seg(int64_t nc, int per_c, int64_t *seg, int32_t *crow, int64_t *coff,
                            int mn) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c <= nc) { seg[c] = c * per_c; coff[c] = c * mn; }
    if (c < nc) crow[c] = 0;
}

int smm_bench(int m, int n, int k, int64_t n_c, int per_c, int n_prm, const SmmParams *prm,
              int reps, double *ms_out, hipStream_t s) {
    if (m < 1 || m > kMaxBlock || n < 1 || n > kMaxBlock || k < 0 || k > kMaxBlock ||
        n_c < 1 || per_c < 1 || n_prm < 1 || reps < 1 || n_c * per_c > (int64_t{1} << 30)) {
        set_error("bench: bad sizes");
        return BSM_EINVAL;
    }
    // k = 0: products cycle through k in {5, 13, 23, 26}
    const int ks_mixed[4] = {5, 13, 23, 26};
    const int nk = k == 0 ? 4 : 1;
    std::vector<int32_t> kval(nk);
    for (int i = 0; i < nk; ++i) kval[i] = k == 0 ? ks_mixed[i] : k;
    const int kmax = *std::max_element(kval.begin(), kval.end());
    const int pool = 1024;
    const int64_t nprod = n_c * per_c;
    // operand pools: A blocks m x k_slot, B blocks k_slot x n
    std::vector<int64_t> aoff(nk * pool + 1), boff(nk * pool + 1);
    std::vector<int32_t> acol(nk * pool);
    for (int sl = 0, t = 0; sl < nk; ++sl)
        for (int q = 0; q < pool; ++q, ++t) {
            aoff[t + 1] = aoff[t] + static_cast<int64_t>(m) * kval[sl];
            boff[t + 1] = boff[t] + static_cast<int64_t>(kval[sl]) * n;
            acol[t] = sl;
        }
    double *av = nullptr, *bv = nullptr, *cv = nullptr, *sq = nullptr, *mx = nullptr;
    int64_t *d_aoff = nullptr, *d_boff = nullptr, *seg = nullptr, *coff = nullptr;
    int32_t *d_acol = nullptr, *d_k = nullptr, *stk_a = nullptr, *stk_b = nullptr;
    int32_t *crow = nullptr, *d_m = nullptr, *d_n = nullptr;
    int *flags = nullptr;
    int st = BSM_OK;
    auto get = [&](auto **p, size_t cnt) { if (st == BSM_OK) st = dalloc(p, cnt, s); };
    get(&av, aoff.back()); get(&bv, boff.back()); get(&cv, n_c * m * n);
    get(&sq, n_c); get(&mx, n_c); get(&d_aoff, aoff.size()); get(&d_boff, boff.size());
    get(&seg, n_c + 1); get(&coff, n_c + 1); get(&d_acol, acol.size()); get(&d_k, nk);
    get(&stk_a, nprod); get(&stk_b, nprod); get(&crow, n_c); get(&d_m, 1); get(&d_n, 1);
    get(&flags, 1);
    std::vector<hipEvent_t> evs;
    if (st == BSM_OK) {
        hipError_t e = hipMemcpyAsync(d_aoff, aoff.data(), sizeof(int64_t) * aoff.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_boff, boff.data(), sizeof(int64_t) * boff.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_acol, acol.data(), sizeof(int32_t) * acol.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_k, kval.data(), sizeof(int32_t) * nk, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_m, &m, sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_n, &n, sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // host vectors die at return
        if (e != hipSuccess) { set_error("bench upload: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st == BSM_OK) {
        k_bench_fill<<<grid_for(aoff.back(), 256), 256, 0, s>>>(av, aoff.back(), 1);
        k_bench_fill<<<grid_for(boff.back(), 256), 256, 0, s>>>(bv, boff.back(), 2);
        k_bench_stack<<<grid_for(nprod, 256), 256, 0, s>>>(nprod, per_c, pool, nk, 3, stk_a, stk_b);
        k_bench_seg<<<grid_for(n_c + 1, 256), 256, 0, s>>>(n_c, per_c, seg, crow, coff, m * n);
        hipError_t e = hipMemsetAsync(flags, 0, sizeof(int), s);
        if (e != hipSuccess) { set_error("bench init: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    SmmArgs a{};
    a.c0 = 0; a.nC = n_c; a.worklist = nullptr; a.seg = seg; a.stk_a = stk_a; a.stk_b = stk_b;
    a.c_row = crow; a.c_col = crow; a.c_blk_off = coff; a.c_vals = cv; a.c_rbs = d_m; a.c_cbs = d_n;
    a.a_col_idx = d_acol; a.a_blk_off = d_aoff; a.a_vals = av; a.k_size = d_k;
    a.b_blk_off = d_boff; a.b_vals = bv; a.alpha = 1.0; a.beta = 0.0;
    a.sq_out = sq; a.mx_out = mx; a.flags = flags;
    a.max_m = m; a.max_n = n; a.max_k = kmax; a.prec = BSM_FP64;
    int64_t *ident = nullptr;
    get(&ident, n_c);
    if (st == BSM_OK) k_bench_iota<<<grid_for(n_c, 256), 256, 0, s>>>(ident, n_c);
    for (int ip = 0; st == BSM_OK && ip < n_prm; ++ip) {
        std::vector<float> t(reps);
        for (int r = 0; st == BSM_OK && r <= reps; ++r) {   // r == 0 warms up
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { st = BSM_EDEVICE; break; }
            evs.push_back(e0); evs.push_back(e1);
            (void)hipEventRecord(e0, s);
            if (prm[ip].family == 2) {
                const int cm = class_of_size(m), cn = class_of_size(n);
                if (cm < 0 || cn < 0 || kmax > 26) { set_error("bench: no class kernel for %dx%d", m, n); st = BSM_EINVAL; break; }
                SmmArgs ca = a;
                ca.worklist = ident;   // the class kernel reads C blocks via the work list
                st = launch_class(ca, 4 * cm + cn, s);
            } else if (prm[ip].family == 3) {
                if (!(m == n && n == k && smm_fixed_available(m, n, k))) {
                    set_error("bench: no compile-time-shape kernel for %dx%dx%d", m, n, k);
                    st = BSM_EINVAL;
                    break;
                }
                SmmArgs fa = a;
                fa.uni_m = m; fa.uni_n = n; fa.uni_k = k;
                const int64_t per = (n_c + kXcds - 1) / kXcds;
                st = launch_fixed(fa, m, static_cast<unsigned>(per * kXcds), s);
            } else {
                st = launch_rt(a, prm[ip], s);
            }
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) { set_error("bench: kernel failed"); st = BSM_EDEVICE; break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t[r - 1] = ms;
        }
        if (st == BSM_OK) {
            std::sort(t.begin(), t.end());
            ms_out[ip] = t[reps / 2];
        }
    }
    for (auto e : evs) (void)hipEventDestroy(e);
    for (void *p : std::initializer_list<void *>{av, bv, cv, sq, mx, d_aoff, d_boff, seg, coff,
                                                d_acol, d_k, stk_a, stk_b, crow, d_m, d_n, flags,
                                                ident})
        dfree(p, s);
    return st;
}

}  // namespace bsm
