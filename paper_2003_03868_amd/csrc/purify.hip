// Density matrix for a fixed occupation N by second-order trace-correcting
// purification (TC2; the density-matrix-based-methods paragraph names it
// among the purifications), which needs no chemical potential:
//   s = ||H||_inf;  X_0 = (s I - H) / (2 s)       (spectrum in [0, 1])
//   k = 0, 1, ...:  Y = filter(X_k X_k)
//                   e_k = (trace X_k - trace Y) / n;  stop if e_k < tol
//                   X_{k+1} = Y if trace X_k > N, else filter(2 X_k - Y)
// Both maps keep [0, 1] and drive every eigenvalue to 0 or 1; the trace test
// steers how many go to 1 towards N.  One multiply per iteration.
#include <cmath>
#include <cstring>

#include "bsm_internal.h"

namespace bsm {

int tc2_purify(Mat &H, double n_occ, const bsm_sign_opts &o, Mat **p_out, bsm_tc2_stats *st,
               hipStream_t s) {
    *p_out = nullptr;
    if (H.nbrows != H.nbcols || H.h_rbs != H.h_cbs) {
        set_error("tc2: H must be square with square diagonal blocks");
        return BSM_EINVAL;
    }
    if (!std::isfinite(n_occ) || !(o.eps_filter >= 0.0) || !std::isfinite(o.eps_filter) ||
        !(o.tol > 0.0) || o.max_iter < 0 || o.max_iter > 120 ||
        (o.norm != BSM_NORM_FROB && o.norm != BSM_NORM_MAXABS)) {
        set_error("tc2: need a finite n_occ, eps_filter >= 0, tol > 0, 0 <= max_iter <= 120, "
                  "a known norm");
        return BSM_EINVAL;
    }
    hipEvent_t t0, t1;
    BSM_HIP(hipEventCreate(&t0));
    BSM_HIP(hipEventCreate(&t1));
    BSM_HIP(hipEventRecord(t0, s));
    const double n = static_cast<double>(H.nrows);
    double sc = 0.0;
    BSM_TRY(inf_norm(H, 0.0, &sc, s));
    st->scale = sc;
    if (!std::isfinite(sc)) { set_error("tc2: H holds NaN or Inf"); return BSM_ENONFINITE; }
    if (sc == 0.0) { set_error("tc2: H is zero"); return BSM_EINVAL; }

    Mat *x = nullptr, *y = nullptr;
    int rc = shift_scale(H, sc, -0.5 / sc, &x, s);                 // (s I - H) / (2 s)
    for (int32_t k = 0; rc == BSM_OK; ++k) {
        rc = alloc_like_sizes(*x, *x, &y, s);
        if (rc != BSM_OK) break;
        bsm_mult_stats ms{};
        rc = multiply(1.0, *x, *x, 0.0, *y, o.eps_filter, o.norm, BSM_FP64, &ms, s);
        if (rc != BSM_OK) break;
        st->n_multiplies++;
        st->flops += ms.flops;
        st->n_products += ms.n_products;
        st->smm_ms += ms.smm_ms;
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
    if (rc == BSM_OK || rc == BSM_ENOCONV) {
        double tp = 0.0;
        const int r2 = trace(*x, &tp, s);
        if (r2 != BSM_OK) { free_mat(x, s); return r2; }
        st->trace_p = tp;
        *p_out = x;
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

}  // namespace bsm
