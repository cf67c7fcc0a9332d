// Error state, the caching device allocator, prefix scan, block offsets and
// the canonical-form check of blocked-CSR matrices.
#include <cstdarg>
#include <cstdio>
#include <map>
#include <mutex>
#include <unordered_map>

#include "bsm_internal.h"

namespace bsm {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }
const char *last_error() { return g_err.c_str(); }

static thread_local std::string g_kernel;
void note_kernel(const char *launch_text) {
    std::string k = launch_text;                    // "(name<args>)" as written
    if (k.size() >= 2 && k.front() == '(' && k.back() == ')') k = k.substr(1, k.size() - 2);
    g_kernel = k;
}
void note_kernelf(const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_kernel = buf;
}
const char *last_kernel() { return g_kernel.c_str(); }

// ----------------------------------------------------------------- memory
// Caching device allocator.  Freed blocks go to a free list of the stream
// they were released on and are handed out again (best fit, at most 1.25x
// the request) to later requests on that stream: stream order makes the
// reuse safe without synchronisation.  hipMalloc runs only when no cached
// block fits; when it fails, cached blocks are returned to the runtime and
// the allocation is retried once.  Sizes are rounded (256 B below 1 MiB,
// 2 MiB above) so similar requests share blocks.

namespace {
struct AllocCache {
    std::mutex mu;
    // (device, stream) -> size -> pointers
    std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>> free_lists;
    std::unordered_map<void *, std::pair<int, size_t>> live;   // ptr -> (device, size)
};
AllocCache &cache() {
    static AllocCache *c = new AllocCache;   // never destroyed: runtime teardown order
    return *c;
}
size_t round_size(size_t b) {
    if (b < (size_t{1} << 20)) return (b + 255) & ~size_t{255};
    const size_t g = size_t{2} << 20;
    return (b + g - 1) / g * g;
}
}  // namespace

static void release_cached(int dev) {
    AllocCache &c = cache();
    std::vector<void *> victims;
    for (auto &kv : c.free_lists) {
        if (kv.first.first != dev) continue;
        for (auto &e : kv.second) victims.push_back(e.second);
        kv.second.clear();
    }
    if (victims.empty()) return;
    (void)hipDeviceSynchronize();
    for (void *p : victims) {
        c.live.erase(p);
        (void)hipFree(p);
    }
}

int dalloc_bytes(void **p, size_t bytes, hipStream_t s) {
    int dev = 0;
    BSM_HIP(hipGetDevice(&dev));
    const size_t want = round_size(bytes == 0 ? 256 : bytes);
    AllocCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto &fl = c.free_lists[{dev, s}];
    auto it = fl.lower_bound(want);
    if (it != fl.end() && it->first <= want + want / 4) {
        *p = it->second;
        fl.erase(it);
        return BSM_OK;
    }
    *p = nullptr;
    hipError_t e = hipMalloc(p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_cached(dev);
        e = hipMalloc(p, want);
    }
    if (e != hipSuccess || *p == nullptr) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        *p = nullptr;
        return BSM_ENOMEM;
    }
    c.live[*p] = {dev, want};
    return BSM_OK;
}

void dfree(void *p, hipStream_t s) {
    if (!p) return;
    AllocCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;   // not ours
    c.free_lists[{it->second.first, s}].emplace(it->second.second, p);
}

void free_mat_arrays(Mat &m, hipStream_t s) {
    dfree(m.row_ptr, s); dfree(m.col_idx, s); dfree(m.blk_off, s); dfree(m.values, s);
    m.row_ptr = nullptr; m.col_idx = nullptr; m.blk_off = nullptr; m.values = nullptr;
    m.nnzb = 0; m.nvalues = 0;
}

void free_mat(Mat *m, hipStream_t s) {
    if (!m) return;
    free_mat_arrays(*m, s);
    dfree(m->rbs, s); dfree(m->cbs, s); dfree(m->roff, s); dfree(m->coff, s);
    delete m;
}

// ------------------------------------------------------------------- scan
// Three-phase exclusive scan: per-tile local scan with tile sums, a scan of
// the tile sums (recursively), then the tile offsets are added.

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    int64_t x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wid] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_tiles(const int64_t *in, int64_t *out, int64_t *tile_sums, int64_t n) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t local = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int64_t i = base + q;
        v[q] = (i < n) ? in[i] : 0;
        local += v[q];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(local, &total);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int64_t i = base + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int64_t *out, const int64_t *tile_off, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / kScanTile];
}

__global__ void k_scan_single(const int64_t *in, int64_t *out, int64_t n) {
    // n <= kScanTile: one tile, also writes out[n] = total.
    const int64_t base = threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t local = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int64_t i = base + q;
        v[q] = (i < n) ? in[i] : 0;
        local += v[q];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(local, &total);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int64_t i = base + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) out[n] = total;
}

__global__ void k_copy_i64(const int64_t *src, int64_t *dst) { *dst = *src; }

// Workspace words of a scan of n values: the tile sums of every level.
int64_t scan_ws_words(int64_t n) {
    int64_t w = 0;
    while (n > kScanTile) {
        const int64_t tiles = (n + kScanTile - 1) / kScanTile;
        w += tiles + 1;
        n = tiles;
    }
    return w;
}

// The scan with its tile sums in ws (scan_ws_words(n) words): kernels only,
// so it can be captured into a graph.
int scan_i64_ws(const int64_t *in, int64_t *out, int64_t n, int64_t *ws, hipStream_t s) {
    if (n <= kScanTile) {
        k_scan_single<<<1, kScanThreads, 0, s>>>(in, out, n);
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    int64_t *sums = ws;
    k_scan_tiles<<<static_cast<unsigned>(tiles), kScanThreads, 0, s>>>(in, out, sums, n);
    BSM_HIP(hipGetLastError());
    BSM_TRY(scan_i64_ws(sums, sums, tiles, ws + tiles + 1, s));   // sums[tiles] = total
    k_scan_add<<<grid_for(n, 256), 256, 0, s>>>(out, sums, n);
    k_copy_i64<<<1, 1, 0, s>>>(sums + tiles, out + n);             // out[n] = total
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    const int64_t w = scan_ws_words(n);
    if (w == 0) return scan_i64_ws(in, out, n, nullptr, s);
    int64_t *ws = nullptr;
    BSM_TRY(dalloc(&ws, w, s));
    const int st = scan_i64_ws(in, out, n, ws, s);
    dfree(ws, s);
    return st;
}

// --------------------------------------------------------- block offsets

__global__ void k_block_sizes(const int64_t *row_ptr, const int32_t *col_idx,
                              const int32_t *rbs, const int32_t *cbs, int32_t nbrows,
                              int64_t *sizes) {
    const int32_t i = blockIdx.x;
    if (i >= nbrows) return;
    const int64_t m = rbs[i];
    for (int64_t t = row_ptr[i] + threadIdx.x; t < row_ptr[i + 1]; t += blockDim.x)
        sizes[t] = m * cbs[col_idx[t]];
}

int compute_blk_off(Mat &m, hipStream_t s) {
    if (m.blk_off == nullptr) BSM_TRY(dalloc(&m.blk_off, m.nnzb + 1, s));
    if (m.nnzb > 0) {
        k_block_sizes<<<m.nbrows, 128, 0, s>>>(m.row_ptr, m.col_idx, m.rbs, m.cbs, m.nbrows,
                                                m.blk_off);
        BSM_HIP(hipGetLastError());
    }
    return scan_i64(m.blk_off, m.blk_off, m.nnzb, s);
}

// ------------------------------------------------------------- validation

__global__ void k_validate(const int64_t *row_ptr, const int32_t *col_idx, int32_t nbrows,
                           int32_t nbcols, int64_t nnzb, int *bad) {
    const int32_t i = blockIdx.x;
    if (i >= nbrows) return;
    const int64_t s = row_ptr[i], e = row_ptr[i + 1];
    if (threadIdx.x == 0) {
        if (i == 0 && s != 0) atomicOr(bad, 1);
        if (e < s || e > nnzb || s < 0) atomicOr(bad, 2);
        if (i == nbrows - 1 && e != nnzb) atomicOr(bad, 4);
    }
    if (e < s || e > nnzb || s < 0) return;
    for (int64_t t = s + threadIdx.x; t < e; t += blockDim.x) {
        const int32_t c = col_idx[t];
        if (c < 0 || c >= nbcols) atomicOr(bad, 8);
        if (t > s && col_idx[t - 1] >= c) atomicOr(bad, 16);
    }
}

int validate_pattern(const Mat &m, hipStream_t s) {
    int *d_bad = nullptr;
    BSM_TRY(dalloc(&d_bad, 1, s));
    BSM_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), s));
    if (m.nbrows > 0) {
        k_validate<<<m.nbrows, 128, 0, s>>>(m.row_ptr, m.col_idx, m.nbrows, m.nbcols, m.nnzb,
                                            d_bad);
        BSM_HIP(hipGetLastError());
    }
    int bad = 0;
    BSM_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    BSM_HIP(hipStreamSynchronize(s));
    dfree(d_bad, s);
    if (bad) {
        set_error("matrix is not canonical blocked CSR (flags 0x%x: 1 row_ptr[0]!=0, "
                  "2 row_ptr decreasing/out of range, 4 row_ptr[nbrows]!=nnzb, "
                  "8 col_idx out of range, 16 col_idx not strictly increasing)", bad);
        return BSM_EINVAL;
    }
    return BSM_OK;
}

}  // namespace bsm
