// Density matrix for a fixed occupation N without a chemical potential, by
// the two purifications the density-matrix-based-methods paragraph names
// besides the sign function.  Both start from
//   s = ||H||_inf;  X_0 = (s I - H) / (2 s)       (spectrum in [0, 1])
// and stop at k when e_k = (trace X_k - trace Y) / n < tol, Y = filter(X_k X_k).
//
// TC2 (second-order trace-correcting), one multiply per iteration:
//   X_{k+1} = Y if trace X_k > N, else filter(2 X_k - Y)
// Both maps keep [0, 1] and drive every eigenvalue to 0 or 1; the trace test
// steers how many go to 1 towards N.
//
// TRS4 (fourth-order trace-resetting), three multiplies per iteration:
//   F = filter(Y filter(4 X_k - 3 Y))     = X^2 (4X - 3X^2)
//   G = filter(D D), D = filter(X_k - Y)  = X^2 (I - X)^2
//   gamma = (N - trace F) / trace G  (0 when the filter has removed all of G)
//   X_{k+1} = filter(2 X_k - Y) if gamma > 6;  Y if gamma < 0;  filter(F + gamma G) otherwise
// F + gamma G fixes 0 and 1 with zero slope for every gamma and, by the
// choice of gamma, resets the trace to N; it keeps [0, 1] only for gamma in
// [0, 6], outside which the TC2 map that moves the trace the right way runs.
#include <cmath>
#include <cstring>

#include "bsm_internal.h"

namespace bsm {

namespace {

// Checks, s = ||H||_inf and X_0 = (s I - H) / (2 s).
int purify_start(const char *what, Mat &H, double n_occ, const bsm_sign_opts &o,
                 bsm_tc2_stats *st, Mat **x, hipStream_t s) {
    if (H.nbrows != H.nbcols || H.h_rbs != H.h_cbs) {
        set_error("%s: H must be square with square diagonal blocks", what);
        return BSM_EINVAL;
    }
    if (!std::isfinite(n_occ) || !(o.eps_filter >= 0.0) || !std::isfinite(o.eps_filter) ||
        !(o.tol > 0.0) || o.max_iter < 0 || o.max_iter > 120 ||
        (o.norm != BSM_NORM_FROB && o.norm != BSM_NORM_MAXABS)) {
        set_error("%s: need a finite n_occ, eps_filter >= 0, tol > 0, 0 <= max_iter <= 120, "
                  "a known norm", what);
        return BSM_EINVAL;
    }
    double sc = 0.0;
    BSM_TRY(inf_norm(H, 0.0, &sc, s));
    st->scale = sc;
    if (!std::isfinite(sc)) { set_error("%s: H holds NaN or Inf", what); return BSM_ENONFINITE; }
    if (sc == 0.0) { set_error("%s: H is zero", what); return BSM_EINVAL; }
    return shift_scale(H, sc, -0.5 / sc, x, s);
}

// out = filter(A B) into a new matrix, FP64 products; accumulates the record.
int product(Mat &A, Mat &B, const bsm_sign_opts &o, Mat **out, bsm_tc2_stats *st,
            hipStream_t s) {
    Mat *c = nullptr;
    BSM_TRY(alloc_like_sizes(A, B, &c, s));
    bsm_mult_stats ms{};
    const int rc = multiply(1.0, A, B, 0.0, *c, o.eps_filter, o.norm, BSM_FP64, &ms, s);
    if (rc != BSM_OK) { free_mat(c, s); return rc; }
    st->n_multiplies++;
    st->flops += ms.flops;
    st->n_products += ms.n_products;
    st->smm_ms += ms.smm_ms;
    *out = c;
    return BSM_OK;
}

// trace(P) of the result, device time, and the result handed out or freed.
int purify_finish(int rc, Mat *x, Mat **p_out, bsm_tc2_stats *st, hipEvent_t t0, hipEvent_t t1,
                  hipStream_t s) {
    if (rc == BSM_OK || rc == BSM_ENOCONV) {
        double tp = 0.0;
        const int r2 = trace(*x, &tp, s);
        if (r2 != BSM_OK) {
            free_mat(x, s);
            rc = r2;
        } else {
            st->trace_p = tp;
            *p_out = x;
        }
    } else {
        free_mat(x, s);
    }
    (void)hipEventRecord(t1, s);
    (void)hipEventSynchronize(t1);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t0, t1) == hipSuccess) st->device_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return rc;
}

}  // namespace

int tc2_purify(Mat &H, double n_occ, const bsm_sign_opts &o, Mat **p_out, bsm_tc2_stats *st,
               hipStream_t s) {
    *p_out = nullptr;
    hipEvent_t t0, t1;
    BSM_HIP(hipEventCreate(&t0));
    BSM_HIP(hipEventCreate(&t1));
    BSM_HIP(hipEventRecord(t0, s));
    const double n = static_cast<double>(H.nrows);
    Mat *x = nullptr, *y = nullptr;
    int rc = purify_start("tc2", H, n_occ, o, st, &x, s);
    for (int32_t k = 0; rc == BSM_OK; ++k) {
        rc = product(*x, *x, o, &y, st, s);
        if (rc != BSM_OK) break;
        double tx = 0.0, ty = 0.0;
        rc = trace(*x, &tx, s);
        if (rc == BSM_OK) rc = trace(*y, &ty, s);
        if (rc != BSM_OK) break;
        const double e = (tx - ty) / n;
        st->e_hist[k] = e;
        st->iterations = k;
        if (!std::isfinite(e)) {
            set_error("tc2: idempotency error is not finite at iteration %d", k);
            rc = BSM_ENONFINITE;
            break;
        }
        if (e < o.tol) break;
        if (k >= o.max_iter) { set_error("tc2: max_iter reached"); rc = BSM_ENOCONV; break; }
        if (tx > n_occ) {                                           // X <- X^2
            st->branch[k] = 0;
            free_mat(x, s);
            x = y;
            y = nullptr;
        } else {                                                    // X <- 2X - X^2
            st->branch[k] = 1;
            Mat *xn = nullptr;
            rc = add_mat(2.0, *x, -1.0, y, 0.0, o.eps_filter, o.norm, &xn, s);
            free_mat(y, s);
            y = nullptr;
            if (rc != BSM_OK) break;
            free_mat(x, s);
            x = xn;
        }
    }
    free_mat(y, s);
    return purify_finish(rc, x, p_out, st, t0, t1, s);
}

int trs4_purify(Mat &H, double n_occ, const bsm_sign_opts &o, Mat **p_out, bsm_tc2_stats *st,
                hipStream_t s) {
    *p_out = nullptr;
    hipEvent_t t0, t1;
    BSM_HIP(hipEventCreate(&t0));
    BSM_HIP(hipEventCreate(&t1));
    BSM_HIP(hipEventRecord(t0, s));
    const double n = static_cast<double>(H.nrows);
    Mat *x = nullptr, *y = nullptr;
    int rc = purify_start("trs4", H, n_occ, o, st, &x, s);
    for (int32_t k = 0; rc == BSM_OK; ++k) {
        rc = product(*x, *x, o, &y, st, s);                         // Y = X^2
        if (rc != BSM_OK) break;
        double tx = 0.0, ty = 0.0;
        rc = trace(*x, &tx, s);
        if (rc == BSM_OK) rc = trace(*y, &ty, s);
        if (rc != BSM_OK) break;
        const double e = (tx - ty) / n;
        st->e_hist[k] = e;
        st->iterations = k;
        if (!std::isfinite(e)) {
            set_error("trs4: idempotency error is not finite at iteration %d", k);
            rc = BSM_ENONFINITE;
            break;
        }
        if (e < o.tol) break;
        if (k >= o.max_iter) { set_error("trs4: max_iter reached"); rc = BSM_ENOCONV; break; }
        Mat *w = nullptr, *f = nullptr, *d = nullptr, *g = nullptr, *xn = nullptr;
        rc = add_mat(4.0, *x, -3.0, y, 0.0, o.eps_filter, o.norm, &w, s);      // 4X - 3Y
        if (rc == BSM_OK) rc = product(*y, *w, o, &f, st, s);                   // F
        if (rc == BSM_OK) rc = add_mat(1.0, *x, -1.0, y, 0.0, o.eps_filter, o.norm, &d, s);
        if (rc == BSM_OK) rc = product(*d, *d, o, &g, st, s);                   // G
        free_mat(w, s);
        free_mat(d, s);
        double tf = 0.0, tg = 0.0;
        if (rc == BSM_OK) rc = trace(*f, &tf, s);
        if (rc == BSM_OK) rc = trace(*g, &tg, s);
        if (rc == BSM_OK) {
            const double gamma = tg > 0.0 ? (n_occ - tf) / tg : 0.0;
            st->gamma_hist[k] = gamma;
            if (gamma > 6.0) {                                                  // X <- 2X - X^2
                st->branch[k] = 1;
                rc = add_mat(2.0, *x, -1.0, y, 0.0, o.eps_filter, o.norm, &xn, s);
            } else if (gamma < 0.0) {                                           // X <- X^2
                st->branch[k] = 0;
                xn = y;
                y = nullptr;
            } else {                                                            // X <- F + gamma G
                st->branch[k] = 2;
                rc = add_mat(1.0, *f, gamma, g, 0.0, o.eps_filter, o.norm, &xn, s);
            }
        }
        free_mat(y, s);
        y = nullptr;
        free_mat(f, s);
        free_mat(g, s);
        if (rc != BSM_OK) { free_mat(xn, s); break; }
        free_mat(x, s);
        x = xn;
    }
    free_mat(y, s);
    return purify_finish(rc, x, p_out, st, t0, t1, s);
}

}  // namespace bsm
