// Newton-Schulz sign iteration driving the block-sparse multiply.
//
// Sign-Method section: sign(A) = A (A^2)^{-1/2} (Eq. signdef); the density
// matrix is P = (I - sign(S^{-1}K - mu I)) S^{-1}/2, here with S = I; after
// every product the result is filtered.  The second-order iteration is the
// refinement function f_1(Z) = Z(3 - Y)/2 of the OT/IR paragraph with
// Y = Z^2, written as X <- 1.5 X - 0.5 X (X X) so that each update is one
// multiply with alpha = -0.5, beta = 1.5 on top of the square Y.
//
// The spectrum is first scaled into [-1, 1] by the infinity norm (a
// Gershgorin bound), so every eigenvalue converges monotonically to +-1.
//
// Orders 3 and 5 (the Pade-type iterations of the Sign-Method section; the
// fifth-order one is Eq. fifth_order_sign, with four multiplies per
// iteration) use the same square Y and residual, then (every product
// filtered):
//   3:  W = 3 Y Y + (15 I - 10 Y);  X' = X W / 8              (f_2 of OT/IR)
//   5:  Y2 = Y Y;  V = 35 Y2 - 180 Y + 378 I;  U = Y2 V + (315 I - 420 Y);
//       X' = X U / 128
//   7:  Y2 = Y Y;  Y3 = Y Y2;  V = (231 Y3 - 1638 Y2 - 8580 I) + 5005 Y;
//       C0 = 9009 Y2 - 6006 Y + 3003 I;  U = Y3 V + C0;  X' = X U / 1024
// where the constant-plus-Y term enters the multiply as its C_in.  The
// section names a seventh-order iteration without printing it; its
// polynomial is the member of the printed family with g'(x) proportional to
// (1 - x^2)^6 and g(1) = 1, evaluated in the Paterson-Stockmeyer split
// q = (3003 - 6006 Y + 9009 Y^2) + Y^3 (231 Y^3 - 1638 Y^2 + 5005 Y - 8580).
//
// Graphs (opts.use_graph = 1): with uniform block sizes that have an FP64
// group kernel (or mixed sizes in {5, 13, 23, 26} with the one-launch
// paired-group kernel asked for), iterations run from graphs of the whole
// device-sized
// multiply (symbolic phase included; graph_iter.hip), captured after an FP64
// iteration on the normal path whose update grew X's block count by at most
// half, and re-captured with larger buffers after an overflow.  Otherwise
// (use_graph = 2 always) the pattern-keyed replay below.
//
// Graph replay (pattern-keyed): once an update leaves the block pattern of X
// unchanged, the symbolic results of both multiplies stay valid for the next
// iteration as long as the filter keeps the same blocks.  The numeric kernels
// of the square (with the residual reduction) and of the update are then
// captured into hipGraphs -- one pair per parity of two ping-pong value
// buffers of X -- and replayed with one wait per iteration.  The replayed
// multiplies check on the device that the filter's keep-set is unchanged; if
// it is not, the (exact) unfiltered product of the replay is filtered and
// compacted anew and the iteration continues on the normal path, so results
// equal those of the normal path.  NaN/Inf in a replayed update sends the
// iteration back to the intact previous iterate, to be redone normally.
#include <cmath>
#include <cstring>

#include "graph_iter.h"
#include "plan.h"

namespace bsm {

static int validate_opts(const Mat &H, const bsm_sign_opts &o) {
    if (H.nbrows != H.nbcols) { set_error("sign: H must be square in blocks"); return BSM_EINVAL; }
    if (H.h_rbs != H.h_cbs) { set_error("sign: H needs square diagonal blocks"); return BSM_EINVAL; }
    if (!(o.eps_filter >= 0.0) || !std::isfinite(o.eps_filter)) { set_error("sign: eps_filter must be finite and >= 0"); return BSM_EINVAL; }
    if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) { set_error("sign: tol must be finite and >= 0"); return BSM_EINVAL; }
    if (o.max_iter < 0 || o.max_iter > 120 || o.fixed_iters < 0 || o.fixed_iters > 120) {
        set_error("sign: max_iter and fixed_iters must be in [0, 120]");
        return BSM_EINVAL;
    }
    if (o.norm != BSM_NORM_FROB && o.norm != BSM_NORM_MAXABS) { set_error("sign: unknown norm"); return BSM_EINVAL; }
    if (o.prec != BSM_FP64 && o.prec != BSM_FP32 && o.prec != BSM_SPLIT_BF16 &&
        o.prec != BSM_SPLIT_BF16X3) {
        set_error("sign: unknown precision");
        return BSM_EINVAL;
    }
    if (o.fp64_final_iters < 0) { set_error("sign: fp64_final_iters must be >= 0"); return BSM_EINVAL; }
    if (o.use_graph < 0 || o.use_graph > 2) { set_error("sign: use_graph must be 0, 1 or 2"); return BSM_EINVAL; }
    if (o.order != 2 && o.order != 3 && o.order != 5 && o.order != 7) {
        set_error("sign: order must be 2, 3, 5 or 7");
        return BSM_EINVAL;
    }
    if (!(o.eps_screen >= 0.0) || !std::isfinite(o.eps_screen)) {
        set_error("sign: eps_screen must be finite and >= 0");
        return BSM_EINVAL;
    }
    if (o.eps_screen > 0.0 && (o.order != 2 || o.prec != BSM_FP64)) {
        set_error("sign: product screening needs order 2 and FP64 products");
        return BSM_EINVAL;
    }
    return BSM_OK;
}

// Precision of the products of iteration k: reduced until the residual first
// drops below prec_switch_tol (with fixed_iters: for all but the last
// fp64_final_iters updates), FP64 afterwards.
static int prec_of(const bsm_sign_opts &o, const bsm_sign_stats &st, int k) {
    if (o.prec == BSM_FP64) return BSM_FP64;
    if (o.fixed_iters > 0) return k < o.fixed_iters - o.fp64_final_iters ? o.prec : BSM_FP64;
    for (int j = 0; j < k; ++j)
        if (st.r_hist[j] < o.prec_switch_tol) return BSM_FP64;
    return o.prec;
}

enum { kGoOn = 0, kStop = 1, kStopNoConv = 2 };

// Stopping rule after r_k is known (stall counts non-decreasing residuals).
static int decide(const bsm_sign_opts &o, const bsm_sign_stats &st, int k, double r, int *stall) {
    if (o.fixed_iters > 0) return k == o.fixed_iters ? kStop : kGoOn;
    if (r < o.tol) return kStop;
    if (k > 0 && r >= st.r_hist[k - 1]) {
        if (++*stall >= 3) {
            set_error("sign: residual stopped decreasing at %g (iteration %d)", r, k);
            return kStopNoConv;
        }
    } else {
        *stall = 0;
    }
    if (k == o.max_iter) {
        set_error("sign: no convergence to %g in %d iterations (r = %g)", o.tol, k, r);
        return kStopNoConv;
    }
    return kGoOn;
}

namespace {
// Device status of a replayed iteration, read back with one copy.
struct Status {
    double d;        // ||Y - I||_F^2
    int32_t f_sq;    // flags of the square
    int32_t f_up;    // flags of the update
    int32_t diff;    // pattern comparison
    int32_t pad_[3];
};

struct Replay {
    hipStream_t s = nullptr;
    bool on = false;
    int prec = 0;
    MulPlan *psq = nullptr, *pup = nullptr;
    double *xbuf[2] = {nullptr, nullptr};   // X's values alternate between these
    int p = 0;                               // X->values == xbuf[p]
    hipGraphExec_t gsq[2] = {nullptr, nullptr}, gup[2] = {nullptr, nullptr};
    double *part = nullptr;                  // per-block-row residual partial sums
    Status *stat = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool up_pending = false;
    int64_t *snap_rp = nullptr;              // pattern of X before the update
    int32_t *snap_ci = nullptr;
    int64_t snap_nnzb = -1, snap_cap = 0;

    void drop_plans() {
        free_plan(psq); psq = nullptr;
        free_plan(pup); pup = nullptr;
    }
    // Leave replay mode; X keeps the buffer it points at.
    void leave(Mat &X) {
        if (!on) return;
        (void)hipStreamSynchronize(s);
        for (int q = 0; q < 2; ++q) {
            if (gsq[q]) (void)hipGraphExecDestroy(gsq[q]);
            if (gup[q]) (void)hipGraphExecDestroy(gup[q]);
            gsq[q] = gup[q] = nullptr;
        }
        for (double *b : xbuf)
            if (b && b != X.values) dfree(b, s);
        xbuf[0] = xbuf[1] = nullptr;
        on = false;
        up_pending = false;
        drop_plans();
    }
    ~Replay() {
        drop_plans();
        dfree(part, s); dfree(stat, s); dfree(snap_rp, s); dfree(snap_ci, s);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Capture the kernels body() queues on a private stream into an executable graph.
template <class F>
int capture(F body, hipGraphExec_t *out) {
    hipStream_t cs = nullptr;
    BSM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        set_error("sign: graph capture: %s", hipGetErrorString(e));
        return BSM_EDEVICE;
    }
    const int rc = body(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (rc == BSM_OK && e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc != BSM_OK) return rc;
    if (e != hipSuccess) { set_error("sign: graph capture: %s", hipGetErrorString(e)); return BSM_EDEVICE; }
    return BSM_OK;
}
}  // namespace

// Keep a copy of X's block pattern (before an update).
static int snapshot(Replay &R, const Mat &X, hipStream_t s) {
    if (X.nnzb > R.snap_cap || !R.snap_rp) {
        dfree(R.snap_ci, s);
        R.snap_ci = nullptr;
        R.snap_cap = 0;
        BSM_TRY(dalloc(&R.snap_ci, X.nnzb + 1, s));
        R.snap_cap = X.nnzb + 1;
        if (!R.snap_rp) BSM_TRY(dalloc(&R.snap_rp, X.nbrows + 1, s));
    }
    BSM_HIP(hipMemcpyAsync(R.snap_rp, X.row_ptr, sizeof(int64_t) * (X.nbrows + 1),
                           hipMemcpyDeviceToDevice, s));
    if (X.nnzb)
        BSM_HIP(hipMemcpyAsync(R.snap_ci, X.col_idx, sizeof(int32_t) * X.nnzb,
                               hipMemcpyDeviceToDevice, s));
    R.snap_nnzb = X.nnzb;
    return BSM_OK;
}

// After an update with retained plans: if X's pattern did not change, capture
// the replay graphs and switch to replay mode; otherwise drop the plans.
static int maybe_enter(Replay &R, Mat &X, Mat &Y, int prec, hipStream_t s) {
    bool same = (X.nnzb == R.snap_nnzb) && R.psq->nval == Y.nvalues && R.pup->nval == X.nvalues &&
                R.psq->a_nval == X.nvalues;
    if (same) {
        BSM_TRY(pattern_differs(R.snap_rp, R.snap_ci, X.row_ptr, X.col_idx, X.nbrows, X.nnzb,
                                &R.stat->diff, s));
        Status h{};
        BSM_HIP(hipMemcpyAsync(&h, R.stat, sizeof(Status), hipMemcpyDeviceToHost, s));
        BSM_HIP(hipStreamSynchronize(s));
        same = (h.diff == 0);
    }
    if (!same) {
        R.drop_plans();
        return BSM_OK;
    }
    double *other = nullptr;
    BSM_TRY(dalloc(&other, X.nvalues, s));
    int rc = zero_flag(&R.stat->f_sq, s);
    if (rc == BSM_OK) rc = zero_flag(&R.stat->f_up, s);
    if (rc != BSM_OK) { dfree(other, s); return rc; }
    R.xbuf[0] = X.values;
    R.xbuf[1] = other;
    R.p = 0;
    for (int q = 0; q < 2 && rc == BSM_OK; ++q) {
        X.values = R.xbuf[q];
        double *next = R.xbuf[1 - q];
        rc = capture([&](hipStream_t cs) -> int {
            BSM_TRY(zero_flag(&R.stat->f_sq, cs));
            BSM_TRY(replay_multiply(*R.psq, X, X, nullptr, Y.values, &R.stat->f_sq, cs));
            return sqdist_identity_dev(Y, 1.0, R.part, &R.stat->d, cs);
        }, &R.gsq[q]);
        if (rc != BSM_OK) break;
        rc = capture([&](hipStream_t cs) -> int {
            BSM_TRY(zero_flag(&R.stat->f_up, cs));
            return replay_multiply(*R.pup, X, Y, &X, next, &R.stat->f_up, cs);
        }, &R.gup[q]);
    }
    X.values = R.xbuf[0];
    R.on = true;            // leave() cleans up what was made
    R.prec = prec;
    if (rc != BSM_OK) R.leave(X);
    return rc;
}

// X <- X q(Y) / d for orders 3, 5 and 7 (see the top of this file); Y = X^2.
static int higher_order_update(const bsm_sign_opts &o, int prec, Mat &X, Mat &Y,
                               bsm_sign_stats *st, hipStream_t s) {
    auto mult = [&](double alpha, Mat &A, Mat &B, double beta, Mat &C) -> int {
        bsm_mult_stats ms{};
        const int rc = multiply(alpha, A, B, beta, C, o.eps_filter, o.norm, prec, &ms, s);
        st->n_multiplies++;
        st->flops += ms.flops;
        st->n_products += ms.n_products;
        st->smm_launches += ms.smm_launches;
        st->smm_ms += ms.smm_ms;
        for (int b = 0; b < 16; ++b) st->class_ms[b] += ms.class_ms[b];
        return rc;
    };
    Mat *c = nullptr, *y2 = nullptr, *v = nullptr, *y3 = nullptr, *v1 = nullptr;
    int rc = BSM_OK;
    if (o.order == 7) {
        rc = alloc_like_sizes(Y, Y, &y2, s);
        if (rc == BSM_OK) rc = mult(1.0, Y, Y, 0.0, *y2);            // Y2
        if (rc == BSM_OK) rc = alloc_like_sizes(Y, Y, &y3, s);
        if (rc == BSM_OK) rc = mult(1.0, Y, *y2, 0.0, *y3);          // Y3
        if (rc == BSM_OK)                                            // 231 Y3 - 1638 Y2 - 8580 I
            rc = add_mat(231.0, *y3, -1638.0, y2, -8580.0, o.eps_filter, o.norm, &v1, s);
        if (rc == BSM_OK) rc = add_mat(1.0, *v1, 5005.0, &Y, 0.0, o.eps_filter, o.norm, &v, s);
        if (rc == BSM_OK)                                            // 9009 Y2 - 6006 Y + 3003 I
            rc = add_mat(9009.0, *y2, -6006.0, &Y, 3003.0, o.eps_filter, o.norm, &c, s);
        if (rc == BSM_OK) rc = mult(1.0, *y3, *v, 1.0, *c);          // U = Y3 V + C0
        if (rc == BSM_OK) rc = mult(1.0 / 1024.0, X, *c, 0.0, X);    // X U / 1024
    } else if (o.order == 3) {
        rc = shift_scale(Y, 1.5, -10.0, &c, s);                      // 15 I - 10 Y
        if (rc == BSM_OK) rc = mult(3.0, Y, Y, 1.0, *c);             // W = 3 Y Y + C
        if (rc == BSM_OK) rc = mult(0.125, X, *c, 0.0, X);           // X W / 8
    } else {
        rc = alloc_like_sizes(Y, Y, &y2, s);
        if (rc == BSM_OK) rc = mult(1.0, Y, Y, 0.0, *y2);            // Y2
        if (rc == BSM_OK)
            rc = add_mat(35.0, *y2, -180.0, &Y, 378.0, o.eps_filter, o.norm, &v, s);
        if (rc == BSM_OK) rc = shift_scale(Y, 0.75, -420.0, &c, s);  // 315 I - 420 Y
        if (rc == BSM_OK) rc = mult(1.0, *y2, *v, 1.0, *c);          // U = Y2 V + C
        if (rc == BSM_OK) rc = mult(1.0 / 128.0, X, *c, 0.0, X);     // X U / 128
    }
    free_mat(c, s);
    free_mat(y2, s);
    free_mat(v, s);
    free_mat(y3, s);
    free_mat(v1, s);
    return rc;
}

int sign_iterate(Mat &H, double mu, const bsm_sign_opts &o, Mat **x_out, bsm_sign_stats *st,
                 hipStream_t s) {
    *x_out = nullptr;
    BSM_TRY(validate_opts(H, o));
    if (!std::isfinite(mu)) { set_error("sign: mu must be finite"); return BSM_EINVAL; }
    hipEvent_t t0, t1;
    BSM_HIP(hipEventCreate(&t0));
    BSM_HIP(hipEventCreate(&t1));
    BSM_HIP(hipEventRecord(t0, s));
    const double n = static_cast<double>(H.nrows);

    double scale = 0.0;
    int rc = inf_norm(H, mu, &scale, s);
    if (rc != BSM_OK) return rc;
    st->scale = scale;
    if (!std::isfinite(scale)) { set_error("sign: H holds NaN or Inf"); return BSM_ENONFINITE; }
    if (scale == 0.0) { set_error("sign: H - mu I is zero"); return BSM_ENOCONV; }

    Mat *X = nullptr, *Y = nullptr;
    BSM_TRY(shift_scale(H, mu, 1.0 / scale, &X, s));
    rc = alloc_like_sizes(*X, *X, &Y, s);
    if (rc != BSM_OK) { free_mat(X, s); return rc; }

    // graphs replay the symbolic results, which screening makes value-dependent
    const bool dev_graph = o.use_graph == 1 && o.order == 2 && o.eps_screen == 0.0 &&
                           graph_iter_ok(*X);
    const bool want_graph = o.use_graph != 0 && !dev_graph && o.order == 2 && o.eps_screen == 0.0;
    GraphIter *G = dev_graph ? gi_create(s, o.eps_filter, o.norm) : nullptr;
    struct GiGuard {
        GraphIter *g;
        ~GiGuard() { gi_destroy(g); }
    } gi_guard{G};
    Replay R;
    R.s = s;
    if (want_graph) {
        rc = dalloc(&R.part, X->nbrows, s);
        if (rc == BSM_OK) rc = dalloc(&R.stat, 1, s);
        for (int i = 0; i < 4 && rc == BSM_OK; ++i)
            if (hipEventCreate(&R.ev[i]) != hipSuccess) { set_error("sign: event creation failed"); rc = BSM_EDEVICE; }
        if (rc != BSM_OK) { free_mat(X, s); free_mat(Y, s); return rc; }
    }

    int stall = 0;
    int stall_at[128] = {0};   // stall count before the decision of iteration k
    for (int k = 0;;) {
        const int prec = prec_of(o, *st, k);
        st->prec_hist[k] = prec;
        bool have_y = false;   // Y of iteration k already formed from a replay
        bool update_only = false;   // square, r_k and the decision done from the graphs
        MulSizes sz_sq, sz_up;
        if (gi_on(G) && prec != BSM_FP64) {
            rc = gi_leave(G, *X, nullptr);
            if (rc != BSM_OK) break;
        } else if (gi_on(G)) {
            // iteration k from the device-sized graphs
            GiStatus gs{};
            double gms = 0.0;
            rc = gi_square(G, &gs, &gms);
            if (rc != BSM_OK) break;
            if (gs.over || (gs.flags & kFlagNonFinite)) {
                // a buffer was too small (or NaN/Inf): iteration k on the
                // normal path, which re-sizes (or reports the error)
                st->graph_fallbacks++;
                rc = gi_leave(G, *X, nullptr);
                if (rc != BSM_OK) break;
            } else {
                st->n_multiplies++;
                st->flops += gs.flops;
                st->n_products += gs.n_products;
                st->smm_launches += 1;
                st->smm_ms += gms;
                const double r = std::sqrt(gs.d) / n;
                st->r_hist[k] = r;
                st->iterations = k;
                st->nnzb_x_hist[k] = gi_x_nnzb(G);
                st->nnzb_y_hist[k] = gs.nnzb;
                if (!std::isfinite(r)) {
                    set_error("sign: residual is not finite at iteration %d", k);
                    rc = BSM_ENONFINITE;
                    break;
                }
                stall_at[k] = stall;
                const int dcs = decide(o, *st, k, r, &stall);
                if (dcs != kGoOn) { rc = (dcs == kStop) ? BSM_OK : BSM_ENOCONV; break; }
                sz_sq.nnzb_u = gs.nnzb_u;
                sz_sq.nnzb = gs.nnzb;
                sz_sq.nval_u = gs.nval_u;
                sz_sq.nval = gs.nval;
                sz_sq.n_groups = gs.n_groups;
                sz_sq.n_entries = gs.n_entries;
                sz_sq.groups = true;
                GiStatus gu{};
                rc = gi_update(G, &gu, &gms);
                if (rc != BSM_OK) break;
                if (gu.over || (gu.flags & kFlagNonFinite)) {
                    // X_k and Y_k are intact: the update on the normal path
                    st->graph_fallbacks++;
                    rc = gi_leave(G, *X, Y);
                    if (rc != BSM_OK) break;
                    update_only = true;
                } else {
                    st->n_multiplies++;
                    st->flops += gu.flops;
                    st->n_products += gu.n_products;
                    st->smm_launches += 1;
                    st->smm_ms += gms;
                    st->graph_replays++;
                    ++k;
                    continue;
                }
            }
        }
        if (R.on) {
            // numeric-only iteration from the captured graphs
            const bool same_prec = (prec == R.prec);
            if (same_prec) {
                (void)hipEventRecord(R.ev[0], s);
                if (hipGraphLaunch(R.gsq[R.p], s) != hipSuccess) { set_error("sign: graph launch failed"); rc = BSM_EDEVICE; break; }
                (void)hipEventRecord(R.ev[1], s);
            }
            Status h{};
            if (hipMemcpyAsync(&h, R.stat, sizeof(Status), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("sign: reading the replay status failed");
                rc = BSM_EDEVICE;
                break;
            }
            float ms = 0.f;
            const bool had_up = R.up_pending;
            if (had_up && hipEventElapsedTime(&ms, R.ev[2], R.ev[3]) == hipSuccess) st->smm_ms += ms;
            R.up_pending = false;
            if (had_up && (h.f_up & kFlagNonFinite)) {
                // NaN/Inf in the replayed update of iteration k-1: back to
                // X_{k-1} and redo k-1 on the normal path (which reports it)
                st->n_multiplies -= 2;
                st->flops -= R.psq->flops + R.pup->flops;
                st->n_products -= R.psq->nprod + R.pup->nprod;
                st->smm_launches -= static_cast<int32_t>(R.psq->ops.size() + R.pup->ops.size());
                st->graph_replays--;
                st->graph_fallbacks++;
                R.p ^= 1;
                X->values = R.xbuf[R.p];
                R.leave(*X);
                --k;
                stall = stall_at[k];
                continue;
            }
            if (had_up && h.f_up) {
                // X_k's product is exact but its filter keeps other blocks:
                // filter it anew; iteration k then runs on the normal path
                double *old = X->values;
                rc = refilter(*R.pup, R.pup->compacted ? R.pup->c_vals_u : old, *X, s);
                for (double *&b : R.xbuf)
                    if (b == old) b = nullptr;   // released with X's old arrays
                st->graph_fallbacks++;
                R.leave(*X);
                if (rc != BSM_OK) break;
            } else if (same_prec && h.f_sq == kFlagPattern) {
                // the square is exact but its filter keeps other blocks
                if (hipEventElapsedTime(&ms, R.ev[0], R.ev[1]) == hipSuccess) st->smm_ms += ms;
                st->n_multiplies++;
                st->flops += R.psq->flops;
                st->n_products += R.psq->nprod;
                st->smm_launches += static_cast<int32_t>(R.psq->ops.size());
                rc = refilter(*R.psq, R.psq->compacted ? R.psq->c_vals_u : Y->values, *Y, s);
                st->graph_fallbacks++;
                R.leave(*X);
                if (rc != BSM_OK) break;
                have_y = true;
            } else if (same_prec && h.f_sq == 0) {
                if (hipEventElapsedTime(&ms, R.ev[0], R.ev[1]) == hipSuccess) st->smm_ms += ms;
                st->n_multiplies++;
                st->flops += R.psq->flops;
                st->n_products += R.psq->nprod;
                st->smm_launches += static_cast<int32_t>(R.psq->ops.size());
                const double r = std::sqrt(h.d) / n;
                st->r_hist[k] = r;
                st->iterations = k;
                st->nnzb_x_hist[k] = X->nnzb;
                st->nnzb_y_hist[k] = Y->nnzb;
                if (!std::isfinite(r)) {
                    set_error("sign: residual is not finite at iteration %d", k);
                    rc = BSM_ENONFINITE;
                    break;
                }
                stall_at[k] = stall;
                const int dcs = decide(o, *st, k, r, &stall);
                if (dcs != kGoOn) { rc = (dcs == kStop) ? BSM_OK : BSM_ENOCONV; break; }
                (void)hipEventRecord(R.ev[2], s);
                if (hipGraphLaunch(R.gup[R.p], s) != hipSuccess) { set_error("sign: graph launch failed"); rc = BSM_EDEVICE; break; }
                (void)hipEventRecord(R.ev[3], s);
                R.up_pending = true;
                st->n_multiplies++;
                st->flops += R.pup->flops;
                st->n_products += R.pup->nprod;
                st->smm_launches += static_cast<int32_t>(R.pup->ops.size());
                st->graph_replays++;
                R.p ^= 1;
                X->values = R.xbuf[R.p];
                ++k;
                continue;
            } else {
                // another precision from here on, or NaN/Inf in the square
                if (same_prec) st->graph_fallbacks++;
                R.leave(*X);
            }
        }

        // iteration k on the normal path (retaining plans when graphs are wanted)
        R.drop_plans();
        bsm_mult_stats ms{};
        if (!update_only) {
            if (!have_y) {
                rc = multiply(1.0, *X, *X, 0.0, *Y, o.eps_filter, o.norm, prec, &ms, s,
                              want_graph ? &R.psq : nullptr, o.eps_screen, &sz_sq);
                st->n_multiplies++;
                st->flops += ms.flops;
                st->n_products += ms.n_products;
                st->n_screened += ms.n_screened;
                st->smm_launches += ms.smm_launches;
                st->smm_ms += ms.smm_ms;
                for (int b = 0; b < 16; ++b) st->class_ms[b] += ms.class_ms[b];
            }
            if (rc != BSM_OK && rc != BSM_ENONFINITE) break;
            double d = 0.0;
            if (rc == BSM_OK) rc = sqdist_identity(*Y, 1.0, &d, s);
            if (rc != BSM_OK && rc != BSM_ENONFINITE) break;
            const double r = std::sqrt(d) / n;
            st->r_hist[k] = (rc == BSM_OK) ? r : NAN;
            st->iterations = k;
            st->nnzb_x_hist[k] = X->nnzb;
            st->nnzb_y_hist[k] = Y->nnzb;
            if (rc == BSM_ENONFINITE || !std::isfinite(r)) {
                set_error("sign: residual is not finite at iteration %d", k);
                rc = BSM_ENONFINITE;
                break;
            }
            stall_at[k] = stall;
            const int dcs = decide(o, *st, k, r, &stall);
            if (dcs != kGoOn) { rc = (dcs == kStop) ? BSM_OK : BSM_ENOCONV; break; }
            if (o.order != 2) {
                rc = higher_order_update(o, prec, *X, *Y, st, s);
                if (rc != BSM_OK) break;
                ++k;
                continue;
            }
        }
        if (want_graph && R.psq) {
            rc = snapshot(R, *X, s);
            if (rc != BSM_OK) break;
        }
        const int64_t x_before = X->nnzb;
        rc = multiply(-0.5, *X, *Y, 1.5, *X, o.eps_filter, o.norm, prec, &ms, s,
                      (want_graph && R.psq) ? &R.pup : nullptr, o.eps_screen, &sz_up);
        st->n_multiplies++;
        st->flops += ms.flops;
        st->n_products += ms.n_products;
        st->n_screened += ms.n_screened;
        st->smm_launches += ms.smm_launches;
        st->smm_ms += ms.smm_ms;
        for (int b = 0; b < 16; ++b) st->class_ms[b] += ms.class_ms[b];
        if (rc != BSM_OK) break;
        if (want_graph && R.psq && R.pup) {
            rc = maybe_enter(R, *X, *Y, prec, s);
            if (rc != BSM_OK) break;
        }
        // the device-sized graphs, once X's block count has settled
        if (G && prec == BSM_FP64 && 2 * X->nnzb <= 3 * x_before) {
            rc = gi_enter(G, *X, *Y, sz_sq, sz_up);
            if (rc != BSM_OK) break;
        }
        ++k;
    }
    if (gi_on(G)) {
        const int r2 = gi_leave(G, *X, nullptr);
        if (r2 != BSM_OK) {
            // X's values are still in the pools only: there is no X to hand out
            R.drop_plans();
            free_mat(Y, s);
            free_mat(X, s);
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return r2;
        }
    }
    R.leave(*X);
    R.drop_plans();
    free_mat(Y, s);
    if (rc == BSM_OK || rc == BSM_ENOCONV) {
        double tx = 0.0;
        int r2 = trace(*X, &tx, s);
        if (r2 != BSM_OK) { free_mat(X, s); return r2; }
        st->trace_x = tx;
        st->trace_p = 0.5 * (n - tx);
    }
    st->nnzb_final = X->nnzb;
    (void)hipEventRecord(t1, s);
    (void)hipEventSynchronize(t1);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t0, t1) == hipSuccess) st->device_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    *x_out = X;
    return rc;
}

}  // namespace bsm
