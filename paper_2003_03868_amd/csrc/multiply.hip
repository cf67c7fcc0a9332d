// C = alpha*A*B + beta*C with the norm filter: the device pipeline.
//
//   1. count     per C block row: C blocks, C scalars, products, flops
//   2. scans     row pointers of C and of the product list (device), then one
//                wait to learn the sizes
//   3. pattern   C col_idx / owning row / matching C_in block
//   4. offsets   C block value offsets (device scan)
//   5. per chunk of block rows (bounded product count, like the paper's
//                bounded batches): product stacks (for the quad kernel merged
//                per 2 x 2 group of C blocks, quad.hip), then the block products
//   6. filter    drop blocks failing the norm test and compact (device)
//
// C's old arrays stay alive until everything that reads them is queued, so C
// may be the same handle as A or B.
//
// With a plan requested, the symbolic results (stacks per chunk, sorted work
// lists, the launches, the filter's keep-set and compaction maps) are kept in
// plan-owned memory for numeric-only repetitions (plan.hip).
#include <algorithm>
#include <climits>
#include <vector>

#include "plan.h"
#include "symbolic.h"

namespace bsm {

// Products per chunk: bounds the stack memory (8 bytes per product; about
// 6 for the quads' entry lists), 4 GiB at the default 2^29, which keeps the
// launches few and large (on the sign workload 2^29 ran 4% faster per step
// than 2^27; 2^30 no faster).  BSM_CHUNK_PRODUCTS overrides it (tests use a
// small value to force chunks).
static int64_t chunk_products() {
    const char *e = getenv("BSM_CHUNK_PRODUCTS");
    const long long x = e ? atoll(e) : 0;
    return x > 0 ? static_cast<int64_t>(x) : (int64_t{1} << 29);
}

// Block-product kernel variant; BSM_SMM_VARIANT overrides the default
// (tests and the tuner compare variants).
int smm_variant() {
    const char *e = getenv("BSM_SMM_VARIANT");
    return e ? atoi(e) : kSmmF64Quad;
}

// Work order of the quads: bands of QR row pairs by QC column pairs
// (BSM_QUAD_TILE_ROWS / BSM_QUAD_TILE_COLS; rows 0 keeps row-pair order).
static int quad_tile(const char *name, int dflt) {
    const char *e = getenv(name);
    return e ? atoi(e) : dflt;
}

// Fewest products per C block for the FP64 group kernel.  Its group lists
// cost a symbolic pass and two more host waits, and the operands a group
// shares are few when C blocks have few products: on random 20%-dense
// products of 64-384 block rows (3-15 products per C block, 13 x 13 and
// 23 x 23 blocks) the one-block kernel took 20-35% less time per call, while
// on the sign workload (16 and more) the groups are faster.  Below this
// count the one-block kernel runs, unless BSM_SMM_VARIANT names a kernel or
// screening needs the groups; BSM_QUAD_MIN_REUSE overrides it.
static double quad_min_reuse() {
    const char *e = getenv("BSM_QUAD_MIN_REUSE");
    return e ? atof(e) : 8.0;
}

// Quads for reduced-precision products: BSM_LOWP_QUAD = 1 always, 0 never;
// default for split-BF16 only (for FP32 products the one-block-per-wave
// kernel measured faster).
static bool lowp_quad(int prec) {
    const char *e = getenv("BSM_LOWP_QUAD");
    if (e) return atoi(e) != 0;
    return prec == BSM_SPLIT_BF16 || prec == BSM_SPLIT_BF16X3;
}

// k segments of the group lists' symbolic walk (one workgroup per row group
// and segment, so the serial walk over the merged A rows is nseg times
// shorter): one per 256 block columns of A, at most 8; BSM_QUAD_KSEG
// overrides it (tests force several segments on small matrices).
int32_t quad_ksegments(int32_t nbk) {
    const char *e = getenv("BSM_QUAD_KSEG");
    int32_t v = e ? atoi(e) : nbk / 256;
    if (v > 8 && !e) v = 8;
    if (v > 64) v = 64;
    return v < 1 ? 1 : v;
}

// Kernel family for a chunk with mixed block sizes (uniform sizes keep the
// requested variant).  Default: one launch per (m, n) class when every size
// is in {5, 13, 23, 26} (measured fastest on the 4096-site mixed workload:
// 7.1 s per sign step, against 8.8 s for the paired-group kernel of
// kSmmF64MQuad, whose one persistent launch per multiply shares operands but
// waits at a barrier per entry for products that are small on average),
// else the run-time-shape persistent kernel.
static int mixed_variant(const SmmArgs &a, int requested) {
    const bool uniform = a.uni_m && a.uni_n && a.uni_k;
    if (uniform) return requested;
    if ((requested == kSmmF64Class || requested == kSmmF64MQuad) && !a.fused_ok) return kSmmF64Fused;
    if (requested == kSmmF64Fixed || requested == kSmmF64Quad)
        return a.fused_ok ? kSmmF64Class : kSmmF64Fused;
    return requested;
}

namespace {
struct Events {
    bool on = false;
    hipEvent_t t0{}, t1{};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> smm;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> cls;   // per-class launches
    ~Events() {
        if (!on) return;
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        for (auto &p : smm) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
        for (auto &p : cls) { (void)hipEventDestroy(p.second.first); (void)hipEventDestroy(p.second.second); }
    }
};
struct Scratch {
    hipStream_t s;
    std::vector<void *> ptrs;
    explicit Scratch(hipStream_t st) : s(st) {}
    template <class T>
    int get(T **p, size_t n) {
        int st = dalloc(p, n, s);
        if (st == BSM_OK) ptrs.push_back(*p);
        return st;
    }
    ~Scratch() { for (void *p : ptrs) dfree(p, s); }
};
}  // namespace

static int check_shapes(const Mat &A, const Mat &B, const Mat &C) {
    if (A.nbcols != B.nbrows || C.nbrows != A.nbrows || C.nbcols != B.nbcols) {
        set_error("block grids do not match: A %dx%d, B %dx%d, C %dx%d", A.nbrows, A.nbcols,
                  B.nbrows, B.nbcols, C.nbrows, C.nbcols);
        return BSM_EINVAL;
    }
    if (A.h_cbs != B.h_rbs) { set_error("A column block sizes differ from B row block sizes"); return BSM_EINVAL; }
    if (C.h_rbs != A.h_rbs || C.h_cbs != B.h_cbs) {
        set_error("C block sizes must be A's row sizes by B's column sizes");
        return BSM_EINVAL;
    }
    if (B.nbcols > kMaxBlockCols) {
        set_error("at most %d block columns are supported (got %d)", kMaxBlockCols, B.nbcols);
        return BSM_EINVAL;
    }
    if (A.nnzb >= (int64_t{1} << 31) || B.nnzb >= (int64_t{1} << 31)) {
        set_error("operands with 2^31 or more stored blocks are not supported");
        return BSM_EINVAL;
    }
    return BSM_OK;
}

int multiply(double alpha, Mat &A, Mat &B, double beta, Mat &C, double eps, int norm, int prec,
             bsm_mult_stats *stats, hipStream_t s, MulPlan **plan, double tau, MulSizes *sizes) {
    BSM_TRY(check_shapes(A, B, C));
    if (!(tau >= 0.0) || !std::isfinite(tau)) { set_error("eps_screen must be finite and >= 0"); return BSM_EINVAL; }
    if (tau > 0.0 && (prec != BSM_FP64 || plan)) {
        set_error("product screening needs FP64 products and no retained plan");
        return BSM_EINVAL;
    }
    if (!(eps >= 0.0) || !std::isfinite(eps)) { set_error("eps_filter must be finite and >= 0"); return BSM_EINVAL; }
    if (norm != BSM_NORM_FROB && norm != BSM_NORM_MAXABS) { set_error("unknown norm %d", norm); return BSM_EINVAL; }
    if (prec != BSM_FP64 && prec != BSM_FP32 && prec != BSM_SPLIT_BF16 && prec != BSM_SPLIT_BF16X3) {
        set_error("unknown precision %d", prec);
        return BSM_EINVAL;
    }
    if (!std::isfinite(alpha) || !std::isfinite(beta)) { set_error("alpha and beta must be finite"); return BSM_EINVAL; }

    const int32_t nbr = A.nbrows;
    const bool use_c = (beta != 0.0) && C.nnzb > 0;
    const int64_t cin_nnzb = C.nnzb;
    Events ev;
    if (stats) {
        ev.on = true;
        BSM_HIP(hipEventCreate(&ev.t0));
        BSM_HIP(hipEventCreate(&ev.t1));
        BSM_HIP(hipEventRecord(ev.t0, s));
    }
    Scratch tmp(s);
    MulPlan *pl = plan ? new MulPlan : nullptr;
    if (pl) pl->s = s;
    // buffers the plan keeps (plan mode) or that die with this call
    auto keep_buf = [&](auto **ptr, size_t n) -> int {
        if (!pl) return tmp.get(ptr, n);
        const int r = dalloc(ptr, n, s);
        if (r == BSM_OK) pl->owned.push_back(*ptr);
        return r;
    };
    struct PlanGuard {
        MulPlan *&p;
        ~PlanGuard() { free_plan(p); }
    } plan_guard{pl};

    SymArgs sa{};
    sa.nbrows = nbr; sa.nbcols = B.nbcols;
    sa.a_row_ptr = A.row_ptr; sa.a_col_idx = A.col_idx;
    sa.b_row_ptr = B.row_ptr; sa.b_col_idx = B.col_idx;
    sa.k_size = A.cbs; sa.c_rbs = A.rbs; sa.c_cbs = B.cbs;
    sa.use_c = use_c ? 1 : 0;
    sa.c_in_row_ptr = use_c ? C.row_ptr : nullptr;
    sa.c_in_col_idx = use_c ? C.col_idx : nullptr;

    // 1-2. counts and scans
    int64_t *c_row_ptr = nullptr, *c_nval = nullptr, *p_row_ptr = nullptr;
    double *flops_row = nullptr;
    BSM_TRY(dalloc(&c_row_ptr, nbr + 1, s));      // becomes the new C's row_ptr
    int st = tmp.get(&c_nval, nbr + 1);
    if (st == BSM_OK) st = tmp.get(&p_row_ptr, nbr + 1);
    if (st == BSM_OK) st = tmp.get(&flops_row, nbr + 1);
    if (st == BSM_OK) st = sym_count(sa, c_row_ptr, c_nval, p_row_ptr, flops_row, s);
    if (st == BSM_OK) st = scan_i64(c_row_ptr, c_row_ptr, nbr, s);
    if (st == BSM_OK) st = scan_i64(c_nval, c_nval, nbr, s);
    if (st == BSM_OK) st = scan_i64(p_row_ptr, p_row_ptr, nbr, s);
    std::vector<int64_t> h_crp(nbr + 1), h_prp(nbr + 1);
    std::vector<double> h_flops(nbr);
    int64_t nval_c = 0;
    if (st == BSM_OK) {
        hipError_t e = hipMemcpyAsync(h_crp.data(), c_row_ptr, sizeof(int64_t) * (nbr + 1), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h_prp.data(), p_row_ptr, sizeof(int64_t) * (nbr + 1), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && nbr) e = hipMemcpyAsync(h_flops.data(), flops_row, sizeof(double) * nbr, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&nval_c, c_nval + nbr, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { set_error("multiply: reading sizes failed: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st != BSM_OK) { dfree(c_row_ptr, s); return st; }
    const int64_t nnzb_c = h_crp[nbr];
    const int64_t nprod = h_prp[nbr];
    double flops = 0.0;
    for (double f : h_flops) flops += f;

    // 3-4. pattern and value offsets of the new C
    Mat nc;
    nc.nbrows = nbr; nc.nbcols = B.nbcols; nc.rbs = A.rbs; nc.cbs = B.cbs;
    nc.row_ptr = c_row_ptr;
    nc.nnzb = nnzb_c;
    nc.nvalues = nval_c;
    int32_t *c_row = nullptr;
    int64_t *cin_map = nullptr;
    double *sq = nullptr, *mx = nullptr;
    int *flags = nullptr;
    st = dalloc(&nc.col_idx, nnzb_c, s);
    if (st == BSM_OK) st = dalloc(&nc.values, nval_c, s);
    if (st == BSM_OK) st = keep_buf(&c_row, nnzb_c);
    if (st == BSM_OK && use_c) st = keep_buf(&cin_map, nnzb_c);
    if (st == BSM_OK) st = keep_buf(&sq, nnzb_c);
    if (st == BSM_OK) st = keep_buf(&mx, nnzb_c);
    if (st == BSM_OK) st = tmp.get(&flags, 1);
    if (st == BSM_OK) {
        hipError_t e = hipMemsetAsync(flags, 0, sizeof(int), s);
        if (e != hipSuccess) { set_error("memset: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st == BSM_OK) st = sym_pattern(sa, c_row_ptr, nc.col_idx, c_row, cin_map, s);
    if (st == BSM_OK) st = compute_blk_off(nc, s);

    // 5. tiled work order, then chunks of whole row bands with a bounded
    //    number of products
    const int rb = tile_rows();
    const int variant = smm_variant();
    int64_t *worklist = nullptr, *worklist2 = nullptr;
    if (st == BSM_OK) st = keep_buf(&worklist, nnzb_c);
    if (st == BSM_OK) st = keep_buf(&worklist2, nnzb_c);  // target of the work-list sorts
    if (st == BSM_OK) st = tile_order(c_row_ptr, nc.col_idx, nbr, B.nbcols, rb, worklist, s);
    // mixed sizes in {5, 13, 23, 26}: groups over paired rows and columns
    // (FP64, no screening), unless another kernel variant is asked for
    const bool mixed_sizes = !(A.uni_r && A.uni_c && B.uni_c);
    bool mixed_ok = true;
    for (const auto *v : {&A.h_rbs, &A.h_cbs, &B.h_cbs})
        for (int32_t b : *v)
            if (b != 5 && b != 13 && b != 23 && b != 26) mixed_ok = false;
    const bool use_mquad = prec == BSM_FP64 && tau == 0.0 && mixed_sizes && mixed_ok &&
                           variant == kSmmF64MQuad;
    std::vector<int32_t> cuts{0};
    {
        // whole row bands; a step that is a multiple of 4 keeps the row
        // groups of the group kernel (2 or 4 rows) in one chunk, one of
        // kPairBand the paired rows of the mixed-size groups
        const int64_t lim = chunk_products();
        const int step = use_mquad ? (rb + kPairBand - 1) / kPairBand * kPairBand : (rb + 3) / 4 * 4;
        int32_t r0 = 0;
        while (r0 < nbr) {
            int32_t r1 = std::min(nbr, r0 + step);
            while (r1 < nbr && h_prp[std::min(nbr, r1 + step)] - h_prp[r0] <= lim)
                r1 = std::min(nbr, r1 + step);
            cuts.push_back(r1);
            r0 = r1;
        }
    }
    int64_t max_p = 0, max_c = 0;
    for (size_t q = 0; q + 1 < cuts.size(); ++q) {
        max_p = std::max(max_p, h_prp[cuts[q + 1]] - h_prp[cuts[q]]);
        max_c = std::max(max_c, h_crp[cuts[q + 1]] - h_crp[cuts[q]]);
    }
    // the quad kernel serves uniform sizes with a compile-time shape unless
    // the tuning table picks another kernel family for them
    bool use_quad = false;
    if (prec == BSM_FP64 && variant == kSmmF64Quad && A.uni_r && A.uni_c && B.uni_c &&
        smm_quad_available(A.uni_r, B.uni_c, A.uni_c)) {
        SmmParams tp;
        use_quad = !(table_lookup(A.uni_r, B.uni_c, A.uni_c, &tp) && tp.family != 3);
        if (use_quad && tau == 0.0 && !getenv("BSM_SMM_VARIANT") &&
            static_cast<double>(nprod) < quad_min_reuse() * static_cast<double>(nnzb_c))
            use_quad = false;
    }
    // reduced precision: quads where they pay, unless another kernel
    // variant is asked for
    if (prec != BSM_FP64 && variant == kSmmF64Quad && lowp_quad(prec) && A.uni_r && A.uni_c &&
        B.uni_c && smm_lowp_available(A.uni_r, B.uni_c, A.uni_c))
        use_quad = true;
    // group shape: quads, or other shapes on request (FP64 only); screening
    // runs through the quads' product masks
    int GR = 2, GC = 2;
    if (use_quad && prec == BSM_FP64 && tau == 0.0) quad_shape(A.uni_r, &GR, &GC);
    if (st == BSM_OK && tau > 0.0 && !use_quad) {
        set_error("product screening needs uniform block sizes 5, 6, 13, 23, 26 or 32 and the "
                  "default kernel variant");
        st = BSM_EINVAL;
    }
    // squared block norms of the operands, and the count of kept products
    double *a_sq = nullptr, *b_sq = nullptr;
    unsigned long long *kept = nullptr;
    if (st == BSM_OK && tau > 0.0) {
        st = tmp.get(&a_sq, A.nnzb);
        if (st == BSM_OK) st = block_sqnorms(A, a_sq, s);
        if (st == BSM_OK && &A != &B) st = tmp.get(&b_sq, B.nnzb);
        if (st == BSM_OK && &A != &B) st = block_sqnorms(B, b_sq, s);
        if (&A == &B) b_sq = a_sq;
        if (st == BSM_OK) st = tmp.get(&kept, 1);
        if (st == BSM_OK) {
            hipError_t e = hipMemsetAsync(kept, 0, sizeof(unsigned long long), s);
            if (e != hipSuccess) { set_error("memset: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
        }
    }
    const int NE = (GR + GC + 3) / 4;                        // int4 per group entry

    // pair maps of the mixed-size groups (host-built, copied to the device)
    MixedPairs mp;
    int32_t *d_rg = nullptr, *d_cgrp = nullptr, *d_cslot = nullptr, *d_cmap = nullptr;
    unsigned long long *mq_counter = nullptr;
    if (st == BSM_OK && use_mquad) {
        mixed_pairs(A.h_rbs, B.h_cbs, &mp);
        st = keep_buf(&d_rg, mp.rg.size());
        if (st == BSM_OK) st = keep_buf(&d_cgrp, mp.cgrp.size());
        if (st == BSM_OK) st = keep_buf(&d_cslot, mp.cslot.size());
        if (st == BSM_OK) st = keep_buf(&d_cmap, mp.cmap.size());
        if (st == BSM_OK) st = keep_buf(&mq_counter, 1);
        hipError_t e = hipSuccess;
        auto up = [&](int32_t *d, const std::vector<int32_t> &h) {
            if (e == hipSuccess && !h.empty())
                e = hipMemcpyAsync(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, s);
        };
        if (st == BSM_OK) { up(d_rg, mp.rg); up(d_cgrp, mp.cgrp); up(d_cslot, mp.cslot); up(d_cmap, mp.cmap); }
        if (e != hipSuccess) { set_error("pair maps: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }

    // one set of stack buffers reused by every chunk; a plan keeps one per
    // chunk; the group kernels build their own lists
    int64_t *seg = nullptr;
    int32_t *stk_a = nullptr, *stk_b = nullptr;
    const bool groups = use_quad || use_mquad;
    if (st == BSM_OK && !pl && !groups) st = tmp.get(&seg, max_c + 1);
    if (st == BSM_OK && !pl && !groups) st = tmp.get(&stk_a, max_p);
    if (st == BSM_OK && !pl && !groups) st = tmp.get(&stk_b, max_p);

    SmmArgs ma{};
    ma.c_row = c_row; ma.c_col = nc.col_idx; ma.c_blk_off = nc.blk_off; ma.c_vals = nc.values;
    ma.c_rbs = A.rbs; ma.c_cbs = B.cbs;
    ma.a_col_idx = A.col_idx; ma.a_blk_off = A.blk_off; ma.a_vals = A.values; ma.k_size = A.cbs;
    ma.b_blk_off = B.blk_off; ma.b_vals = B.values;
    ma.cin_map = cin_map;
    ma.cin_blk_off = use_c ? C.blk_off : nullptr;
    ma.cin_vals = use_c ? C.values : nullptr;
    ma.alpha = alpha; ma.beta = beta;
    ma.sq_out = sq; ma.mx_out = mx; ma.flags = flags;
    ma.max_m = A.max_rbs; ma.max_n = B.max_cbs; ma.max_k = A.max_cbs;
    ma.uni_m = A.uni_r; ma.uni_n = B.uni_c; ma.uni_k = A.uni_c;
    {
        auto in_set = [](const std::vector<int32_t> &v) {
            for (int32_t b : v)
                if (b != 5 && b != 13 && b != 23 && b != 26) return false;
            return true;
        };
        ma.fused_ok = (in_set(A.h_rbs) && in_set(A.h_cbs) && in_set(B.h_cbs)) ? 1 : 0;
    }
    ma.prec = prec;
    ma.seg = seg; ma.stk_a = stk_a; ma.stk_b = stk_b;
    ma.worklist = worklist;
    if (st == BSM_OK) st = keep_buf(&ma.counter, 1);         // persistent kernels' counter

    if (st == BSM_OK && prec != BSM_FP64) {
        if (!(A.uni_r && A.uni_c && B.uni_c && smm_lowp_available(A.uni_r, B.uni_c, A.uni_c))) {
            set_error("reduced-precision products need uniform block sizes 5, 13, 23, 26 or 32");
            st = BSM_EINVAL;
        }
        uint32_t *apk = nullptr, *bpk = nullptr;
        if (st == BSM_OK) st = keep_buf(&apk, lowp_words(A.nvalues, prec));
        if (st == BSM_OK) st = pack_lowp(A.values, A.nvalues, apk, prec, s);
        if (st == BSM_OK && &A != &B) {
            st = keep_buf(&bpk, lowp_words(B.nvalues, prec));
            if (st == BSM_OK) st = pack_lowp(B.values, B.nvalues, bpk, prec, s);
        } else {
            bpk = apk;
        }
        ma.a_pk = apk;
        ma.b_pk = bpk;
        ma.a_pk_n = A.nvalues;
        ma.b_pk_n = B.nvalues;
        if (pl) { pl->apk = apk; pl->bpk = bpk; }
    }

    int32_t n_launch = 0;
    int64_t sum_groups = 0, sum_entries = 0;
    auto launch = [&](const MulOp &op) -> int {
        ++n_launch;
        const int r = run_op(op, s);
        if (r == BSM_OK && pl) pl->ops.push_back(op);
        return r;
    };

    for (size_t q = 0; st == BSM_OK && q + 1 < cuts.size(); ++q) {
        const int32_t r0 = cuts[q], r1 = cuts[q + 1];
        ma.c0 = h_crp[r0];
        ma.nC = h_crp[r1] - h_crp[r0];
        if (ma.nC == 0) continue;
        if (groups) {
            // groups of this chunk's C blocks and their merged entry lists;
            // without a plan the buffers live for this chunk only
            Scratch ctmp(s);
            auto qbuf = [&](auto **ptr, size_t n) -> int { return pl ? keep_buf(ptr, n) : ctmp.get(ptr, n); };
            int32_t g0 = 0;
            int64_t npairs = (static_cast<int64_t>(r1 - r0) + GR - 1) / GR;
            if (use_mquad) {
                g0 = mp.band_g0[r0 / kPairBand];
                npairs = mp.band_g0[(r1 + kPairBand - 1) / kPairBand] - g0;
            }
            int64_t *q_off = nullptr, *q_cblk = nullptr, *e_off = nullptr, *q_order = nullptr,
                    *e_seg = nullptr;
            int32_t *pm = nullptr;
            int32_t *q_col = nullptr;
            int4 *ent = nullptr;
            int64_t nq = 0, ne = 0;
            auto read_total = [&](const int64_t *d, int64_t *h) -> int {
                hipError_t e = hipMemcpyAsync(h, d, sizeof(int64_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) { set_error("quads: %s", hipGetErrorString(e)); return BSM_EDEVICE; }
                return BSM_OK;
            };
            QuadSymArgs qa{};
            qa.r0 = r0; qa.r1 = r1; qa.nbcols = B.nbcols; qa.gr = GR; qa.gc = GC;
            qa.nseg = quad_ksegments(A.nbcols);
            qa.kseg = (A.nbcols + qa.nseg - 1) / qa.nseg;
            if (qa.kseg < 1) qa.kseg = 1;
            qa.a_row_ptr = A.row_ptr; qa.a_col_idx = A.col_idx;
            qa.b_row_ptr = B.row_ptr; qa.b_col_idx = B.col_idx;
            qa.c_row_ptr = c_row_ptr; qa.c_col_idx = nc.col_idx;
            qa.a_sq = a_sq; qa.b_sq = b_sq; qa.tau2 = tau * tau; qa.kept = kept;
            if (use_mquad) {
                qa.map = 1;
                qa.g0 = g0;
                qa.ngroups = npairs;
                qa.ncg = static_cast<int32_t>(mp.cmap.size() / 2);
                qa.rg = d_rg; qa.cgrp = d_cgrp; qa.cslot = d_cslot; qa.cmap = d_cmap;
            }
            st = qbuf(&q_off, npairs + 1);
            if (st == BSM_OK) st = quad_pairs(qa, q_off, s);
            if (st == BSM_OK) st = scan_i64(q_off, q_off, npairs, s);
            if (st == BSM_OK) st = read_total(q_off + npairs, &nq);
            if (st == BSM_OK) st = qbuf(&q_cblk, static_cast<size_t>(GR) * GC * nq);
            if (st == BSM_OK) st = qbuf(&e_off, nq + 1);
            if (st == BSM_OK && qa.nseg > 1) st = qbuf(&e_seg, static_cast<size_t>(nq) * qa.nseg + 1);
            if (qa.nseg == 1) e_seg = e_off;
            if (st == BSM_OK) st = qbuf(&q_col, nq);
            qa.q_off = q_off;
            qa.q_cblk = q_cblk;
            qa.q_col = q_col;
            qa.e_off = e_seg;
            if (st == BSM_OK) st = quad_stack(qa, false, s);
            const int qr = quad_tile("BSM_QUAD_TILE_ROWS", 0), qc = quad_tile("BSM_QUAD_TILE_COLS", 16);
            if (st == BSM_OK && qr > 0 && nq > 0 && !use_mquad) {
                st = qbuf(&q_order, nq);
                if (st == BSM_OK)
                    st = tile_order(q_off, q_col, static_cast<int32_t>(npairs), (B.nbcols + GC - 1) / GC,
                                    qr, q_order, s, qc);
            }
            const int64_t nsl = nq * qa.nseg;                       // (group, segment) counts
            if (st == BSM_OK) st = scan_i64(e_seg, e_seg, nsl, s);
            if (st == BSM_OK && qa.nseg > 1) st = quad_seg_starts(e_seg, qa.nseg, nq, e_off, s);
            if (st == BSM_OK) st = read_total(e_seg + nsl, &ne);
            if (st == BSM_OK && ne > INT32_MAX) {
                // the fill pass keeps entry offsets inside a row group as int32
                set_error("more than 2^31 group entries in one chunk; lower BSM_CHUNK_PRODUCTS");
                st = BSM_EINVAL;
            }
            sum_groups += nq;
            sum_entries += ne;
            if (st == BSM_OK) st = qbuf(&ent, static_cast<size_t>(ne) * NE);
            if (st == BSM_OK && tau > 0.0) st = qbuf(&pm, ne);
            qa.ent = ent;
            qa.pm = pm;
            if (st == BSM_OK) st = quad_stack(qa, true, s);
            if (st != BSM_OK) break;
            MulOp op;
            op.a = ma;
            op.kind = use_mquad ? kOpMQuad : kOpQuad;
            op.a.counter = use_mquad ? mq_counter : ma.counter;
            op.a.n_quads = nq;
            op.a.q_cblk = q_cblk;
            op.a.q_seg = e_off;
            op.a.q_ent = ent;
            if (st == BSM_OK && use_mquad && nq > 0) {
                int8_t *rank = nullptr;
                st = ctmp.get(&rank, nq);
                if (st == BSM_OK) st = qbuf(&q_order, nq);
                if (st == BSM_OK) st = mquad_order(op.a, rank, q_order, s);
                if (st != BSM_OK) break;
            }
            op.a.q_order = q_order;
            op.a.q_gr = GR;
            op.a.q_gc = GC;
            op.a.q_pm = pm;
            std::pair<hipEvent_t, hipEvent_t> pe{};
            if (ev.on) {
                BSM_HIP(hipEventCreate(&pe.first));
                BSM_HIP(hipEventCreate(&pe.second));
                BSM_HIP(hipEventRecord(pe.first, s));
            }
            st = launch(op);
            if (ev.on) {
                BSM_HIP(hipEventRecord(pe.second, s));
                ev.smm.push_back(pe);
            }
            continue;
        }
        if (pl) {
            const int64_t np = h_prp[r1] - h_prp[r0];
            st = keep_buf(&seg, ma.nC + 1);
            if (st == BSM_OK) st = keep_buf(&stk_a, np);
            if (st == BSM_OK) st = keep_buf(&stk_b, np);
            if (st != BSM_OK) break;
            ma.seg = seg; ma.stk_a = stk_a; ma.stk_b = stk_b;
        }
        st = sym_stack(sa, r0, r1, c_row_ptr, p_row_ptr, seg, stk_a, stk_b, s);
        if (st != BSM_OK) break;

        // mixed sizes: cost-sorted list for the fused persistent launch, or
        // class-sorted list for one launch per (m, n) class
        const int var = (prec == BSM_FP64) ? mixed_variant(ma, variant) : -1;
        int64_t hist[64] = {0};
        if (var == kSmmF64Fused || var == kSmmF64Class) {
            if (worklist2 == nullptr) { set_error("internal: no sort buffer"); st = BSM_EDEVICE; break; }
            st = sort_worklist(worklist, worklist2, ma.c0, ma.nC,
                               var == kSmmF64Fused ? kKeyCost : kKeyClass, c_row, nc.col_idx,
                               A.rbs, B.cbs, seg, var == kSmmF64Class ? hist : nullptr, s);
            if (st != BSM_OK) break;
            ma.worklist = worklist2;
        } else {
            ma.worklist = worklist;
        }
        std::pair<hipEvent_t, hipEvent_t> pe{};
        if (ev.on) {
            BSM_HIP(hipEventCreate(&pe.first));
            BSM_HIP(hipEventCreate(&pe.second));
            BSM_HIP(hipEventRecord(pe.first, s));
        }
        MulOp op;
        op.a = ma;
        if (prec != BSM_FP64) {
            op.kind = kOpLowp;
            st = launch(op);
        } else if (var == kSmmF64Class) {
            int64_t off = 0;
            for (int b = 0; b < 17 && st == BSM_OK; ++b) {
                if (hist[b] == 0) continue;
                op.a.worklist = worklist2 + off;
                op.a.nC = hist[b];
                // per class: the (m, n)-specialised kernel unless the tuning
                // table holds run-time-kernel parameters for (m, n, any k)
                static const int sz[4] = {5, 13, 23, 26};
                SmmParams prm;
                if (b < 16 && !(table_lookup(sz[b / 4], sz[b % 4], 0, &prm) && prm.family != 2)) {
                    op.kind = kOpClass;
                    op.id = b;
                } else if (b < 16) {
                    op.kind = kOpRt;
                    op.prm = prm;
                } else {
                    op.kind = kOpVariant;
                    op.id = kSmmF64Tuned;
                }
                std::pair<hipEvent_t, hipEvent_t> ce{};
                if (ev.on && b < 16) {
                    BSM_HIP(hipEventCreate(&ce.first));
                    BSM_HIP(hipEventCreate(&ce.second));
                    BSM_HIP(hipEventRecord(ce.first, s));
                }
                st = launch(op);
                if (ev.on && b < 16) {
                    BSM_HIP(hipEventRecord(ce.second, s));
                    ev.cls.push_back({b, ce});
                }
                off += hist[b];
            }
        } else {
            op.kind = kOpVariant;
            op.id = var;
            st = launch(op);
        }
        if (ev.on) {
            BSM_HIP(hipEventRecord(pe.second, s));
            ev.smm.push_back(pe);
        }
    }

    // 6. filter
    int64_t nnzb_after = nnzb_c;
    CompactKeep ck;
    if (st == BSM_OK && eps > 0.0)
        st = compact_by_norm(nc, sq, mx, eps, norm, s, &nnzb_after, pl ? &ck : nullptr);
    if (pl) {
        // the plan owns the keep maps and the unfiltered layout
        for (void *q : {static_cast<void *>(ck.kidx), static_cast<void *>(ck.koff),
                        static_cast<void *>(ck.row_ptr), static_cast<void *>(ck.col_idx),
                        static_cast<void *>(ck.blk_off), static_cast<void *>(ck.values)})
            if (q) pl->owned.push_back(q);
        if (st == BSM_OK) {
            pl->compacted = ck.compacted;
            if (ck.compacted) {
                pl->c_row_ptr_u = ck.row_ptr;
                pl->c_col_u = ck.col_idx;
                pl->c_blk_off_u = ck.blk_off;
                pl->c_vals_u = ck.values;
            } else {
                st = keep_buf(&pl->c_col_u, nnzb_c);
                if (st == BSM_OK) st = keep_buf(&pl->c_blk_off_u, nnzb_c + 1);
                if (st == BSM_OK) st = keep_buf(&pl->c_row_ptr_u, nbr + 1);
                hipError_t e = hipSuccess;
                if (st == BSM_OK)
                    e = hipMemcpyAsync(pl->c_row_ptr_u, nc.row_ptr, sizeof(int64_t) * (nbr + 1),
                                       hipMemcpyDeviceToDevice, s);
                if (st == BSM_OK && e == hipSuccess && nnzb_c)
                    e = hipMemcpyAsync(pl->c_col_u, nc.col_idx, sizeof(int32_t) * nnzb_c,
                                       hipMemcpyDeviceToDevice, s);
                if (st == BSM_OK && e == hipSuccess)
                    e = hipMemcpyAsync(pl->c_blk_off_u, nc.blk_off, sizeof(int64_t) * (nnzb_c + 1),
                                       hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) { set_error("plan copy: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
            }
            for (MulOp &o : pl->ops) { o.a.c_col = pl->c_col_u; o.a.c_blk_off = pl->c_blk_off_u; }
        }
    }
    int h_flags = 0;
    if (st == BSM_OK) {
        hipError_t e = hipMemcpyAsync(&h_flags, flags, sizeof(int), hipMemcpyDeviceToHost, s);
        if (ev.on && e == hipSuccess) e = hipEventRecord(ev.t1, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { set_error("multiply: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st != BSM_OK) {
        dfree(nc.row_ptr, s); dfree(nc.col_idx, s); dfree(nc.blk_off, s); dfree(nc.values, s);
        return st;
    }

    // swap the new arrays into C (old ones are freed in stream order)
    free_mat_arrays(C, s);
    C.row_ptr = nc.row_ptr; C.col_idx = nc.col_idx; C.blk_off = nc.blk_off; C.values = nc.values;
    C.nnzb = nc.nnzb; C.nvalues = nc.nvalues;
    C.stream = s;

    if (sizes) {
        sizes->nnzb_u = nnzb_c;
        sizes->nnzb = nnzb_after;
        sizes->nval_u = nval_c;
        sizes->nval = nc.nvalues;
        sizes->n_groups = sum_groups;
        sizes->n_entries = sum_entries;
        sizes->groups = (use_quad && prec == BSM_FP64) || use_mquad;
    }
    if (stats) {
        stats->n_products = nprod;
        stats->flops = flops;
        stats->nnzb_unfiltered = nnzb_c;
        stats->nnzb = nnzb_after;
        stats->smm_launches = n_launch;
        if (tau > 0.0 && kept) {
            unsigned long long h_kept = 0;
            if (hipMemcpyAsync(&h_kept, kept, sizeof(h_kept), hipMemcpyDeviceToHost, s) == hipSuccess &&
                hipStreamSynchronize(s) == hipSuccess)
                stats->n_screened = nprod - static_cast<int64_t>(h_kept);
            // uniform blocks: every product costs the same, so the flops
            // actually done scale with the kept count
            if (nprod > 0) stats->flops = flops * static_cast<double>(h_kept) / static_cast<double>(nprod);
        }
        float ms = 0.f;
        double smm = 0.0;
        for (auto &p : ev.smm) {
            if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) smm += ms;
        }
        stats->smm_ms = smm;
        stats->total_ms = (hipEventElapsedTime(&ms, ev.t0, ev.t1) == hipSuccess) ? ms : 0.0;
        for (int b = 0; b < 16; ++b) stats->class_ms[b] = 0.0;
        for (auto &p : ev.cls)
            if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess)
                stats->class_ms[p.first] += ms;
    }
    if (pl) {
        pl->alpha = alpha; pl->beta = beta; pl->eps = eps; pl->norm = norm; pl->prec = prec;
        pl->use_c = use_c;
        pl->same_ab = (&A == &B);
        pl->a_nnzb = A.nnzb; pl->b_nnzb = B.nnzb; pl->a_nval = A.nvalues; pl->b_nval = B.nvalues;
        pl->cin_nnzb = use_c ? cin_nnzb : 0;
        pl->nnzb_u = nnzb_c; pl->nval_u = nval_c;
        pl->nnzb = nc.nnzb; pl->nval = nc.nvalues;
        pl->flops = flops; pl->nprod = nprod;
        pl->sq = sq; pl->mx = mx;
        pl->kidx = ck.kidx; pl->koff = ck.koff;
    }
    if (h_flags & kFlagNonFinite) {
        set_error("a product block holds NaN or Inf");
        return BSM_ENONFINITE;
    }
    if (pl) { *plan = pl; pl = nullptr; }
    return BSM_OK;
}

}  // namespace bsm
