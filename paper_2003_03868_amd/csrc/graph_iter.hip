// Device-sized Newton-Schulz iterations replayed from captured hipGraphs.
//
// The normal multiply learns its sizes on the host (C blocks and scalars,
// groups, entries) and allocates to fit them, so a whole iteration cannot be
// captured.  Here every size stays in device memory.  Buffers are reserved
// up front with fixed capacities, taken from an iteration run on the normal
// path plus headroom; each kernel reads the counts it needs from device
// memory; and after each scan a capacity check records an overflow in a
// device status word and empties the structure that overflowed, so the
// kernels after it do no work and stay inside their buffers.  One iteration
// (FP64 group kernels: uniform block sizes, or sizes in {5, 13, 23, 26} with
// every (m, n) class in one persistent launch; one chunk) is six graphs:
//
//   square  Y = filter(X X):  symbolic | block products | filter, ||Y - I||^2
//   update  X' = filter(1.5 X - 0.5 X Y):  symbolic | block products | filter
//
// launched with events around the block products and one wait after each
// multiply, where the host reads r_k, the sizes and the flags (the
// Sign-Method iteration needs r_k to stop).  X alternates between two
// buffers, each parity with its own six graphs.  A multiply whose record
// shows an overflow (or NaN/Inf) left its inputs intact; that iteration is
// redone on the normal path, which also yields the sizes to re-size the
// buffers with.  The kernels and their order are those of the normal path
// with a single chunk (the chunks of the normal path only split the group
// list), so the results are the same bits.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "graph_iter.h"
#include "smm.h"
#include "symbolic.h"

namespace bsm {

namespace {

// Headroom of the capacities over the sizes they are taken from
// (BSM_GRAPH_HEADROOM, >= 1).
double headroom() {
    const char *e = getenv("BSM_GRAPH_HEADROOM");
    const double h = e ? atof(e) : 1.25;
    return h >= 1.0 ? h : 1.0;
}

// Multipliers of the capacities (unfiltered C blocks, groups, entries, X, Y;
// the scalar capacities follow their blocks) from BSM_GRAPH_CAPS="c,g,e,x,y"
// (default 1 each; tests use values below 1 to make one buffer too small;
// X keeps room for the current X).
void cap_scales(double (&m)[5]) {
    for (double &v : m) v = 1.0;
    const char *e = getenv("BSM_GRAPH_CAPS");
    for (int i = 0; e && *e && i < 5; ++i) {
        char *end = nullptr;
        const double v = strtod(e, &end);
        if (end == e) break;
        if (v > 0.0) m[i] = v;
        e = (*end == ',') ? end + 1 : end;
    }
}

bool in_mixed_set(const std::vector<int32_t> &v) {
    for (int32_t b : v)
        if (b != 5 && b != 13 && b != 23 && b != 26) return false;
    return true;
}

__global__ void k_gi_reset(GiStatus *st) {
    st->over = 0;
    st->flags = 0;
    st->d = 0.0;
}

// Record an overflow: *total above cap sets `bit`.
__global__ void k_gi_check(const int64_t *total, int64_t cap, int bit, GiStatus *st) {
    if (*total > cap) st->over |= bit;
}

// arr[0 .. n) = 0 when the record holds any of `bits`.
__global__ void k_gi_zero_if(const GiStatus *st, int bits, int64_t *arr, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && (st->over & bits)) arr[i] = 0;
}

// arr[*from * mul .. n) = 0: the counts past the last item.
__global__ void k_gi_zero_from(const int64_t *from, int64_t mul, int64_t *arr, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && i >= *from * mul) arr[i] = 0;
}

// Scalars of every C block (m n), to be scanned into value offsets.
__global__ void k_gi_sizes(const int64_t *rp, const int32_t *col, const int32_t *rbs,
                           const int32_t *cbs, int64_t *sizes) {
    const int32_t i = blockIdx.x;
    const int64_t m = rbs[i];
    for (int64_t t = rp[i] + threadIdx.x; t < rp[i + 1]; t += blockDim.x) sizes[t] = m * cbs[col[t]];
}

// The filter's test for the first *n_dev of cap unfiltered blocks (the test
// of the normal path's compaction) and the kept blocks' scalar counts; 0
// past them.
__global__ void k_gi_keep(const double *sq, const double *mx, const int64_t *bo,
                          const int64_t *n_dev, int64_t cap, double eps, int norm, int64_t *keep,
                          int64_t *ksize) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= cap) return;
    bool k = false;
    if (t < *n_dev) k = (norm == BSM_NORM_MAXABS) ? !(mx[t] < eps) : !(sq[t] < eps * eps);
    keep[t] = k ? 1 : 0;
    ksize[t] = k ? bo[t + 1] - bo[t] : 0;
}

// Filtered row pointers from the keep scan.
__global__ void k_gi_rows(const int64_t *c_rp, const int64_t *kidx, int32_t nbr, int64_t *out_rp) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i <= nbr) out_rp[i] = kidx[c_rp[i]];
}

// One wave per unfiltered block: a kept block to its filtered place.
__global__ void __launch_bounds__(64)
k_gi_compact(const int64_t *kidx, const int64_t *koff, const int64_t *n_dev, const int32_t *col,
             const int64_t *bo, const double *vals, int32_t *out_col, int64_t *out_bo,
             double *out_vals) {
    const int64_t t = blockIdx.x;
    if (t >= *n_dev) return;
    const int64_t d = kidx[t];
    if (kidx[t + 1] == d) return;   // dropped
    const int64_t src = bo[t], len = bo[t + 1] - src, dst = koff[t];
    if (threadIdx.x == 0) {
        out_col[d] = col[t];
        out_bo[d] = dst;
    }
    for (int64_t e = threadIdx.x; e < len; e += 64) out_vals[dst + e] = vals[src + e];
}

// The closing value offset of the filtered matrix.
__global__ void k_gi_bo_end(const int64_t *nkept, const int64_t *nval, int64_t *out_bo) {
    out_bo[*nkept] = *nval;
}

// Sizes into the record; products and flops summed over the block rows (the
// flops are sums of integers below 2^53, so the order does not matter).
__global__ void __launch_bounds__(256)
k_gi_status(const int64_t *c_rp, const int64_t *c_bo, const int64_t *q_off, int64_t nrg,
            const int64_t *e_tot, const int64_t *out_rp, const int64_t *nval,
            const int64_t *p_cnt, const double *fl, int32_t nbr, GiStatus *st) {
    __shared__ int64_t part[256 / kWave];
    __shared__ double partf[256 / kWave];
    int64_t np = 0;
    double f = 0.0;
    for (int32_t i = threadIdx.x; i < nbr; i += 256) {
        np += p_cnt[i];
        f += fl[i];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        np += __shfl_xor(np, o, kWave);
        f += __shfl_xor(f, o, kWave);
    }
    if (threadIdx.x % kWave == 0) {
        part[threadIdx.x / kWave] = np;
        partf[threadIdx.x / kWave] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        double tf = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) {
            t += part[w];
            tf += partf[w];
        }
        st->n_products = t;
        st->flops = tf;
        const int64_t nu = c_rp[nbr];
        st->nnzb_u = nu;
        st->nval_u = c_bo[nu];
        st->n_groups = q_off[nrg];
        st->n_entries = *e_tot;
        st->nnzb = out_rp[nbr];
        st->nval = *nval;
    }
}

// A matrix held in fixed-capacity buffers: cap blocks, vcap scalars.
struct PoolMat {
    int64_t cap = 0, vcap = 0;
    int64_t *rp = nullptr;
    int32_t *ci = nullptr;
    int64_t *bo = nullptr;
    double *v = nullptr;
};

template <class F>
int capture(F body, hipGraphExec_t *out) {
    hipStream_t cs = nullptr;
    BSM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        set_error("graph capture: %s", hipGetErrorString(e));
        return BSM_EDEVICE;
    }
    const int rc = body(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (rc == BSM_OK && e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc != BSM_OK) return rc;
    if (e != hipSuccess) { set_error("graph capture: %s", hipGetErrorString(e)); return BSM_EDEVICE; }
    return BSM_OK;
}

}  // namespace

struct Caps {
    int64_t c = 0, cv = 0, g = 0, e = 0, x = 0, xv = 0, y = 0, yv = 0;
};

struct GraphIter {
    hipStream_t s = nullptr;
    double eps = 0.0;
    int norm = 0;
    bool on = false;          // X lives in x[p] and the graphs are current
    bool have_graphs = false;
    bool off = false;         // the buffers did not fit: iterations stay on the normal path
    int p = 0;
    Mat proto;                // X's sizes (block-size arrays borrowed from X)
    int32_t nbr = 0, nbc = 0, b = 0;   // b: the uniform block size, 0 for mixed sizes
    bool mixed = false;
    int gr = 2, gc = 2;
    int32_t nseg = 1, kseg = 1;
    int64_t nrg = 0;          // row groups
    MixedPairs mp;
    Caps cap;
    int64_t x_nnzb = 0, x_nval = 0, y_nnzb = 0, y_nval = 0;
    std::vector<void *> owned;
    PoolMat x[2], y;
    // mixed sizes: pair maps and the persistent kernel's work order
    int32_t *d_rg = nullptr, *d_cgrp = nullptr, *d_cslot = nullptr, *d_cmap = nullptr;
    unsigned long long *counter = nullptr;
    int8_t *rank = nullptr;
    int64_t *q_order = nullptr;
    // the unfiltered product (shared by the square and the update)
    int64_t *c_rp = nullptr, *c_nval = nullptr, *p_cnt = nullptr, *c_bo = nullptr;
    double *flops_row = nullptr;
    int32_t *c_col = nullptr, *c_row = nullptr;
    int64_t *cin_map = nullptr;
    double *c_vals = nullptr, *sq = nullptr, *mx = nullptr;
    // groups and their entries
    int64_t *q_off = nullptr, *q_cblk = nullptr, *e_seg = nullptr, *e_off = nullptr;
    int32_t *q_col = nullptr;
    int4 *ent = nullptr;
    // filter, scans, residual, records
    int64_t *kidx = nullptr, *koff = nullptr, *ws = nullptr;
    double *part = nullptr;
    GiStatus *st = nullptr;   // [0] square, [1] update
    hipGraphExec_t g[2][6] = {};
    hipEvent_t ev[4] = {};

    template <class T>
    int get(T **ptr, size_t n) {
        const int r = dalloc(ptr, n, s);
        if (r == BSM_OK) owned.push_back(*ptr);
        return r;
    }
    void drop_graphs() {
        for (auto &row : g)
            for (auto &e : row) {
                if (e) (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
        have_graphs = false;
    }
    void release() {
        drop_graphs();
        if (!owned.empty()) (void)hipStreamSynchronize(s);
        for (void *q : owned) dfree(q, s);
        owned.clear();
        cap = Caps{};
    }
    ~GraphIter() {
        release();
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    Mat view(const PoolMat &m) const {
        Mat v = proto;
        v.row_ptr = m.rp;
        v.col_idx = m.ci;
        v.blk_off = m.bo;
        v.values = m.v;
        v.nnzb = 0;
        v.nvalues = 0;
        return v;
    }
    int alloc(const Caps &c);
    int mult_sym(const Mat &A, const Mat &B, bool use_c, GiStatus *rec, hipStream_t cs);
    int mult_smm(const Mat &A, const Mat &B, const Mat *Cin, double alpha, double beta,
                 GiStatus *rec, hipStream_t cs);
    int mult_post(const PoolMat &out, GiStatus *rec, hipStream_t cs);
    int capture_all();
};

bool graph_iter_ok(const Mat &X) {
    if (X.nbrows != X.nbcols || X.nbrows == 0 || X.h_rbs != X.h_cbs) return false;
    if (X.uni_r && X.uni_r == X.uni_c) {
        const int b = X.uni_r;
        if (!smm_quad_available(b, b, b) || smm_variant() != kSmmF64Quad) return false;
        SmmParams tp;
        if (table_lookup(b, b, b, &tp) && tp.family != 3) return false;
        int gr = 2, gc = 2;
        quad_shape(b, &gr, &gc);
        return gr == 2 && gc == 2;
    }
    // mixed sizes: the paired groups in one persistent launch per multiply
    return in_mixed_set(X.h_rbs) && smm_variant() == kSmmF64MQuad;
}

GraphIter *gi_create(hipStream_t s, double eps, int norm) {
    GraphIter *g = new GraphIter;
    g->s = s;
    g->eps = eps;
    g->norm = norm;
    return g;
}

void gi_destroy(GraphIter *g) { delete g; }
bool gi_on(const GraphIter *g) { return g && g->on; }
int64_t gi_x_nnzb(const GraphIter *g) { return g->x_nnzb; }

int GraphIter::alloc(const Caps &c) {
    release();
    const int32_t ne4 = (gr + gc + 3) / 4;
    int r = BSM_OK;
    auto req = [&](auto **ptr, size_t n) {
        if (r == BSM_OK) r = get(ptr, n);
    };
    for (PoolMat *m : {&x[0], &x[1], &y}) {
        m->cap = (m == &y) ? c.y : c.x;
        m->vcap = (m == &y) ? c.yv : c.xv;
        req(&m->rp, nbr + 1);
        req(&m->ci, m->cap);
        req(&m->bo, m->cap + 1);
        req(&m->v, m->vcap);
    }
    req(&c_rp, nbr + 1);
    req(&c_nval, nbr + 1);
    req(&p_cnt, nbr + 1);
    req(&flops_row, nbr + 1);
    req(&c_bo, c.c + 1);
    req(&c_col, c.c);
    req(&c_row, c.c);
    req(&cin_map, c.c);
    req(&c_vals, c.cv);
    req(&sq, c.c);
    req(&mx, c.c);
    req(&q_off, nrg + 1);
    req(&q_cblk, static_cast<size_t>(gr) * gc * c.g);
    req(&q_col, c.g);
    req(&e_seg, static_cast<size_t>(c.g) * nseg + 1);
    if (nseg > 1) req(&e_off, c.g + 1);
    req(&ent, static_cast<size_t>(c.e) * ne4);
    req(&kidx, c.c + 1);
    req(&koff, c.c + 1);
    const int64_t w = std::max({scan_ws_words(nbr), scan_ws_words(nrg),
                                scan_ws_words(c.g * nseg), scan_ws_words(c.c)});
    req(&ws, std::max<int64_t>(w, 1));
    req(&part, nbr);
    req(&st, 2);
    if (mixed) {
        req(&d_rg, mp.rg.size());
        req(&d_cgrp, mp.cgrp.size());
        req(&d_cslot, mp.cslot.size());
        req(&d_cmap, std::max<size_t>(mp.cmap.size(), 1));
        req(&counter, 1);
        req(&rank, c.g);
        req(&q_order, c.g);
    }
    if (r != BSM_OK) { release(); return r; }
    if (nseg == 1) e_off = e_seg;
    if (mixed) {
        hipError_t e = hipSuccess;
        auto up = [&](int32_t *d, const std::vector<int32_t> &h) {
            if (e == hipSuccess && !h.empty())
                e = hipMemcpyAsync(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, s);
        };
        up(d_rg, mp.rg); up(d_cgrp, mp.cgrp); up(d_cslot, mp.cslot); up(d_cmap, mp.cmap);
        if (e != hipSuccess) {
            release();
            set_error("graph iteration: pair maps: %s", hipGetErrorString(e));
            return BSM_EDEVICE;
        }
    }
    cap = c;
    return BSM_OK;
}

// Symbolic part: pattern and value offsets of the unfiltered product, groups
// and their entry lists (the normal path's steps 1-5 for one chunk), with
// capacity checks.
int GraphIter::mult_sym(const Mat &A, const Mat &B, bool use_c, GiStatus *rec, hipStream_t cs) {
    k_gi_reset<<<1, 1, 0, cs>>>(rec);
    SymArgs sa{};
    sa.nbrows = nbr; sa.nbcols = nbc;
    sa.a_row_ptr = A.row_ptr; sa.a_col_idx = A.col_idx;
    sa.b_row_ptr = B.row_ptr; sa.b_col_idx = B.col_idx;
    sa.k_size = A.cbs; sa.c_rbs = A.rbs; sa.c_cbs = B.cbs;
    sa.use_c = use_c ? 1 : 0;
    sa.c_in_row_ptr = use_c ? A.row_ptr : nullptr;   // C_in is X = A
    sa.c_in_col_idx = use_c ? A.col_idx : nullptr;
    BSM_TRY(sym_count(sa, c_rp, c_nval, p_cnt, flops_row, cs));
    BSM_TRY(scan_i64_ws(c_rp, c_rp, nbr, ws, cs));
    k_gi_check<<<1, 1, 0, cs>>>(c_rp + nbr, cap.c, kGiOverC, rec);
    k_gi_zero_if<<<grid_for(nbr + 1, 256), 256, 0, cs>>>(rec, kGiOverC, c_rp, nbr + 1);
    BSM_TRY(sym_pattern(sa, c_rp, c_col, c_row, use_c ? cin_map : nullptr, cs));
    // value offsets; scalars over capacity empty C as well
    k_gi_sizes<<<nbr, 128, 0, cs>>>(c_rp, c_col, A.rbs, B.cbs, c_bo);
    k_gi_zero_from<<<grid_for(cap.c + 1, 256), 256, 0, cs>>>(c_rp + nbr, 1, c_bo, cap.c + 1);
    BSM_TRY(scan_i64_ws(c_bo, c_bo, cap.c, ws, cs));
    k_gi_check<<<1, 1, 0, cs>>>(c_bo + cap.c, cap.cv, kGiOverC, rec);
    k_gi_zero_if<<<grid_for(nbr + 1, 256), 256, 0, cs>>>(rec, kGiOverC, c_rp, nbr + 1);

    QuadSymArgs qa{};
    qa.r0 = 0; qa.r1 = nbr; qa.nbcols = nbc; qa.gr = gr; qa.gc = gc;
    qa.nseg = nseg; qa.kseg = kseg;
    qa.a_row_ptr = A.row_ptr; qa.a_col_idx = A.col_idx;
    qa.b_row_ptr = B.row_ptr; qa.b_col_idx = B.col_idx;
    qa.c_row_ptr = c_rp; qa.c_col_idx = c_col;
    qa.q_off = q_off; qa.q_cblk = q_cblk; qa.q_col = q_col; qa.e_off = e_seg; qa.ent = ent;
    if (mixed) {
        qa.map = 1;
        qa.g0 = 0;
        qa.ngroups = nrg;
        qa.ncg = static_cast<int32_t>(mp.cmap.size() / 2);
        qa.rg = d_rg; qa.cgrp = d_cgrp; qa.cslot = d_cslot; qa.cmap = d_cmap;
    }
    BSM_TRY(quad_pairs(qa, q_off, cs));
    BSM_TRY(scan_i64_ws(q_off, q_off, nrg, ws, cs));
    k_gi_check<<<1, 1, 0, cs>>>(q_off + nrg, cap.g, kGiOverG, rec);
    k_gi_zero_if<<<grid_for(nrg + 1, 256), 256, 0, cs>>>(rec, kGiOverG, q_off, nrg + 1);
    BSM_TRY(quad_stack(qa, false, cs));
    const int64_t nsl = cap.g * nseg;
    k_gi_zero_from<<<grid_for(nsl + 1, 256), 256, 0, cs>>>(q_off + nrg, nseg, e_seg, nsl + 1);
    BSM_TRY(scan_i64_ws(e_seg, e_seg, nsl, ws, cs));
    // entries over capacity: no groups at all from here on
    k_gi_check<<<1, 1, 0, cs>>>(e_seg + nsl, cap.e, kGiOverE, rec);
    k_gi_zero_if<<<grid_for(nrg + 1, 256), 256, 0, cs>>>(rec, kGiOverE, q_off, nrg + 1);
    if (nseg > 1) BSM_TRY(quad_seg_starts(e_seg, nseg, cap.g, e_off, cs));
    BSM_TRY(quad_stack(qa, true, cs));
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// Block products: the group kernel over the device count of groups.
int GraphIter::mult_smm(const Mat &A, const Mat &B, const Mat *Cin, double alpha, double beta,
                        GiStatus *rec, hipStream_t cs) {
    SmmArgs a{};
    a.c_row = c_row; a.c_col = c_col; a.c_blk_off = c_bo; a.c_vals = c_vals;
    a.c_rbs = A.rbs; a.c_cbs = B.cbs;
    a.a_col_idx = A.col_idx; a.a_blk_off = A.blk_off; a.a_vals = A.values; a.k_size = A.cbs;
    a.b_blk_off = B.blk_off; a.b_vals = B.values;
    a.cin_map = Cin ? cin_map : nullptr;
    a.cin_blk_off = Cin ? Cin->blk_off : nullptr;
    a.cin_vals = Cin ? Cin->values : nullptr;
    a.alpha = alpha; a.beta = beta;
    a.sq_out = sq; a.mx_out = mx; a.flags = &rec->flags;
    a.max_m = A.max_rbs; a.max_n = B.max_cbs; a.max_k = A.max_cbs;
    a.uni_m = A.uni_r; a.uni_n = B.uni_c; a.uni_k = A.uni_c;
    a.fused_ok = mixed ? 1 : 0;
    a.prec = BSM_FP64;
    a.counter = counter;
    a.n_quads = cap.g;
    a.n_quads_dev = q_off + nrg;
    a.q_cblk = q_cblk; a.q_seg = e_off; a.q_ent = ent;
    a.q_gr = gr; a.q_gc = gc;
    if (!mixed) return launch_quad(a, cs);
    BSM_TRY(mquad_order(a, rank, q_order, cs));
    a.q_order = q_order;
    return launch_mquad(a, cs);
}

// Filter and compaction into `out`, then the record's sizes.
int GraphIter::mult_post(const PoolMat &out, GiStatus *rec, hipStream_t cs) {
    k_gi_keep<<<grid_for(cap.c, 256), 256, 0, cs>>>(sq, mx, c_bo, c_rp + nbr, cap.c, eps, norm,
                                                   kidx, koff);
    BSM_TRY(scan_i64_ws(kidx, kidx, cap.c, ws, cs));
    BSM_TRY(scan_i64_ws(koff, koff, cap.c, ws, cs));
    k_gi_check<<<1, 1, 0, cs>>>(kidx + cap.c, out.cap, kGiOverOut, rec);
    k_gi_check<<<1, 1, 0, cs>>>(koff + cap.c, out.vcap, kGiOverOut, rec);
    k_gi_zero_if<<<grid_for(cap.c + 1, 256), 256, 0, cs>>>(rec, kGiOverOut, kidx, cap.c + 1);
    k_gi_zero_if<<<grid_for(cap.c + 1, 256), 256, 0, cs>>>(rec, kGiOverOut, koff, cap.c + 1);
    k_gi_rows<<<grid_for(nbr + 1, 256), 256, 0, cs>>>(c_rp, kidx, nbr, out.rp);
    k_gi_compact<<<static_cast<unsigned>(cap.c), 64, 0, cs>>>(kidx, koff, c_rp + nbr, c_col, c_bo,
                                                             c_vals, out.ci, out.bo, out.v);
    k_gi_bo_end<<<1, 1, 0, cs>>>(kidx + cap.c, koff + cap.c, out.bo);
    k_gi_status<<<1, 256, 0, cs>>>(c_rp, c_bo, q_off, nrg, e_seg + cap.g * nseg, out.rp,
                                   koff + cap.c, p_cnt, flops_row, nbr, rec);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int GraphIter::capture_all() {
    drop_graphs();
    for (int q = 0; q < 2; ++q) {
        const Mat X = view(x[q]), Y = view(y);
        // square: Y = filter(X X), then ||Y - I||_F^2
        BSM_TRY(capture([&](hipStream_t cs) { return mult_sym(X, X, false, &st[0], cs); }, &g[q][0]));
        BSM_TRY(capture([&](hipStream_t cs) { return mult_smm(X, X, nullptr, 1.0, 0.0, &st[0], cs); },
                        &g[q][1]));
        BSM_TRY(capture([&](hipStream_t cs) {
            BSM_TRY(mult_post(y, &st[0], cs));
            return sqdist_identity_dev(Y, 1.0, part, &st[0].d, cs);
        }, &g[q][2]));
        // update: X' = filter(-0.5 X Y + 1.5 X) into the other buffer
        BSM_TRY(capture([&](hipStream_t cs) { return mult_sym(X, Y, true, &st[1], cs); }, &g[q][3]));
        BSM_TRY(capture([&](hipStream_t cs) { return mult_smm(X, Y, &X, -0.5, 1.5, &st[1], cs); },
                        &g[q][4]));
        BSM_TRY(capture([&](hipStream_t cs) { return mult_post(x[1 - q], &st[1], cs); }, &g[q][5]));
    }
    have_graphs = true;
    return BSM_OK;
}

// Copy a matrix's pattern, offsets and values into a pool buffer.
static int to_pool(const Mat &m, PoolMat &pm, int32_t nbr, hipStream_t s) {
    BSM_HIP(hipMemcpyAsync(pm.rp, m.row_ptr, sizeof(int64_t) * (nbr + 1), hipMemcpyDeviceToDevice, s));
    BSM_HIP(hipMemcpyAsync(pm.bo, m.blk_off, sizeof(int64_t) * (m.nnzb + 1), hipMemcpyDeviceToDevice, s));
    if (m.nnzb) {
        BSM_HIP(hipMemcpyAsync(pm.ci, m.col_idx, sizeof(int32_t) * m.nnzb, hipMemcpyDeviceToDevice, s));
        BSM_HIP(hipMemcpyAsync(pm.v, m.values, sizeof(double) * m.nvalues, hipMemcpyDeviceToDevice, s));
    }
    return BSM_OK;
}

// Own arrays for m (nnzb blocks, nval scalars) copied from a pool buffer.
static int from_pool(const GraphIter &g, const PoolMat &pm, int64_t nnzb, int64_t nval, Mat &m) {
    hipStream_t s = g.s;
    Mat n;
    int r = dalloc(&n.row_ptr, g.nbr + 1, s);
    if (r == BSM_OK) r = dalloc(&n.col_idx, nnzb, s);
    if (r == BSM_OK) r = dalloc(&n.blk_off, nnzb + 1, s);
    if (r == BSM_OK) r = dalloc(&n.values, nval, s);
    hipError_t e = hipSuccess;
    if (r == BSM_OK) {
        e = hipMemcpyAsync(n.row_ptr, pm.rp, sizeof(int64_t) * (g.nbr + 1), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(n.blk_off, pm.bo, sizeof(int64_t) * (nnzb + 1), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && nnzb)
            e = hipMemcpyAsync(n.col_idx, pm.ci, sizeof(int32_t) * nnzb, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && nval)
            e = hipMemcpyAsync(n.values, pm.v, sizeof(double) * nval, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) { set_error("graph iteration: copy: %s", hipGetErrorString(e)); r = BSM_EDEVICE; }
    }
    if (r != BSM_OK) {
        dfree(n.row_ptr, s); dfree(n.col_idx, s); dfree(n.blk_off, s); dfree(n.values, s);
        return r;
    }
    free_mat_arrays(m, s);
    m.row_ptr = n.row_ptr; m.col_idx = n.col_idx; m.blk_off = n.blk_off; m.values = n.values;
    m.nnzb = nnzb;
    m.nvalues = nval;
    return BSM_OK;
}

int gi_enter(GraphIter *g, Mat &X, Mat &Y, const MulSizes &sq, const MulSizes &up) {
    if (g->on) { set_error("internal: graph iteration entered twice"); return BSM_EINVAL; }
    if (g->off || !sq.groups || !up.groups) return BSM_OK;   // another kernel did the products
    if (!g->proto.rbs) {
        g->proto = X;
        g->proto.row_ptr = nullptr; g->proto.col_idx = nullptr;
        g->proto.blk_off = nullptr; g->proto.values = nullptr;
        g->nbr = X.nbrows; g->nbc = X.nbcols;
        g->mixed = !(X.uni_r && X.uni_r == X.uni_c);
        g->b = g->mixed ? 0 : X.uni_r;
        if (g->mixed) {
            g->gr = g->gc = 2;
            mixed_pairs(X.h_rbs, X.h_cbs, &g->mp);
            g->nrg = g->mp.band_g0.back();
        } else {
            quad_shape(g->b, &g->gr, &g->gc);
            g->nrg = (static_cast<int64_t>(g->nbr) + g->gr - 1) / g->gr;
        }
        g->nseg = quad_ksegments(X.nbcols);
        g->kseg = (X.nbcols + g->nseg - 1) / g->nseg;
        if (g->kseg < 1) g->kseg = 1;
        for (hipEvent_t &e : g->ev)
            if (!e) BSM_HIP(hipEventCreate(&e));
    }
    // capacities: the sizes times the headroom, plus a little slack (none
    // at headroom 1, so that any growth overflows), within the structural
    // bounds, at least 1
    const double h = headroom();
    double m[5];
    cap_scales(m);
    auto grow = [&](int64_t want, int64_t bound, double mult) {
        const double v = std::ceil(static_cast<double>(want) * h * mult) + (h > 1.0 ? 64.0 : 0.0);
        return std::max<int64_t>(1, static_cast<int64_t>(std::min(v, static_cast<double>(bound))));
    };
    const int64_t dense = static_cast<int64_t>(g->nbr) * g->nbc;
    const int64_t dense_v = X.nrows * X.ncols;
    const int64_t ncg = g->mixed ? static_cast<int64_t>(g->mp.cmap.size() / 2)
                                 : (g->nbc + g->gc - 1) / g->gc;
    Caps want;
    want.c = grow(std::max(sq.nnzb_u, up.nnzb_u), dense, m[0]);
    want.cv = grow(std::max(sq.nval_u, up.nval_u), dense_v, m[0]);
    want.g = grow(std::max(sq.n_groups, up.n_groups), g->nrg * ncg, m[1]);
    want.e = grow(std::max(sq.n_entries, up.n_entries), INT32_MAX, m[2]);
    want.x = std::max(X.nnzb, grow(std::max(up.nnzb, X.nnzb), dense, m[3]));
    want.xv = std::max(X.nvalues, grow(std::max(up.nval, X.nvalues), dense_v, m[3]));
    want.y = grow(sq.nnzb, dense, m[4]);
    want.yv = grow(sq.nval, dense_v, m[4]);
    if (want.c > INT32_MAX || std::max({sq.n_entries, up.n_entries}) > INT32_MAX) return BSM_OK;
    const Caps &c = g->cap;
    if (want.c > c.c || want.cv > c.cv || want.g > c.g || want.e > c.e || want.x > c.x ||
        want.xv > c.xv || want.y > c.y || want.yv > c.yv) {
        Caps n;
        n.c = std::max(want.c, c.c); n.cv = std::max(want.cv, c.cv);
        n.g = std::max(want.g, c.g); n.e = std::max(want.e, c.e);
        n.x = std::max(want.x, c.x); n.xv = std::max(want.xv, c.xv);
        n.y = std::max(want.y, c.y); n.yv = std::max(want.yv, c.yv);
        const int r = g->alloc(n);
        if (r == BSM_ENOMEM) {
            // device memory too small for the fixed-capacity buffers: the
            // iterations continue on the normal path, which sizes each
            // multiply to fit
            clear_error();
            g->off = true;
            return BSM_OK;
        }
        BSM_TRY(r);
    }
    if (!g->have_graphs) BSM_TRY(g->capture_all());
    BSM_TRY(to_pool(X, g->x[0], g->nbr, g->s));
    g->x_nnzb = X.nnzb;
    g->x_nval = X.nvalues;
    g->p = 0;
    free_mat_arrays(X, g->s);
    X.nnzb = g->x_nnzb;
    X.nvalues = g->x_nval;
    free_mat_arrays(Y, g->s);
    g->on = true;
    return BSM_OK;
}

static int read_status(GraphIter *g, int which, GiStatus *out, double *smm_ms) {
    BSM_HIP(hipMemcpyAsync(out, &g->st[which], sizeof(GiStatus), hipMemcpyDeviceToHost, g->s));
    BSM_HIP(hipStreamSynchronize(g->s));
    float ms = 0.f;
    *smm_ms = (hipEventElapsedTime(&ms, g->ev[2 * which], g->ev[2 * which + 1]) == hipSuccess) ? ms : 0.0;
    return BSM_OK;
}

static int launch3(GraphIter *g, int first, int which) {
    hipStream_t s = g->s;
    BSM_HIP(hipGraphLaunch(g->g[g->p][first], s));
    BSM_HIP(hipEventRecord(g->ev[2 * which], s));
    BSM_HIP(hipGraphLaunch(g->g[g->p][first + 1], s));
    BSM_HIP(hipEventRecord(g->ev[2 * which + 1], s));
    BSM_HIP(hipGraphLaunch(g->g[g->p][first + 2], s));
    return BSM_OK;
}

int gi_square(GraphIter *g, GiStatus *out, double *smm_ms) {
    BSM_TRY(launch3(g, 0, 0));
    BSM_TRY(read_status(g, 0, out, smm_ms));
    if (!out->over) {
        g->y_nnzb = out->nnzb;
        g->y_nval = out->nval;
    }
    return BSM_OK;
}

int gi_update(GraphIter *g, GiStatus *out, double *smm_ms) {
    BSM_TRY(launch3(g, 3, 1));
    BSM_TRY(read_status(g, 1, out, smm_ms));
    if (!out->over && !(out->flags & kFlagNonFinite)) {
        g->p ^= 1;
        g->x_nnzb = out->nnzb;
        g->x_nval = out->nval;
    }
    return BSM_OK;
}

int gi_leave(GraphIter *g, Mat &X, Mat *Y) {
    if (!g->on) return BSM_OK;
    BSM_TRY(from_pool(*g, g->x[g->p], g->x_nnzb, g->x_nval, X));
    g->on = false;   // X is whole again (else the pools still hold it)
    if (Y) BSM_TRY(from_pool(*g, g->y, g->y_nnzb, g->y_nval, *Y));
    return BSM_OK;
}

}  // namespace bsm
