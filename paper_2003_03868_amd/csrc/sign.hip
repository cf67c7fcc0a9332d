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
#include <cmath>
#include <cstring>

#include "bsm_internal.h"

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
    if (o.prec != BSM_FP64 && o.prec != BSM_FP32 && o.prec != BSM_SPLIT_BF16) { set_error("sign: unknown precision"); return BSM_EINVAL; }
    if (o.fp64_final_iters < 0) { set_error("sign: fp64_final_iters must be >= 0"); return BSM_EINVAL; }
    return BSM_OK;
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

    bool low = (o.prec != BSM_FP64);
    int stall = 0;
    for (int k = 0;; ++k) {
        // precision of this round's products
        int prec = BSM_FP64;
        if (low) {
            if (o.fixed_iters > 0) low = (k < o.fixed_iters - o.fp64_final_iters);
            else if (k > 0 && st->r_hist[k - 1] < o.prec_switch_tol) low = false;
            if (low) prec = o.prec;
        }
        st->prec_hist[k] = prec;
        bsm_mult_stats ms{};
        rc = multiply(1.0, *X, *X, 0.0, *Y, o.eps_filter, o.norm, prec, &ms, s);
        st->n_multiplies++;
        st->flops += ms.flops;
        st->n_products += ms.n_products;
        st->smm_ms += ms.smm_ms;
        if (rc != BSM_OK && rc != BSM_ENONFINITE) break;
        double d = 0.0;
        if (rc == BSM_OK) rc = sqdist_identity(*Y, 1.0, &d, s);
        if (rc != BSM_OK && rc != BSM_ENONFINITE) break;
        const double r = std::sqrt(d) / n;
        st->r_hist[k] = (rc == BSM_OK) ? r : NAN;
        st->iterations = k;
        if (rc == BSM_ENONFINITE || !std::isfinite(r)) {
            set_error("sign: residual is not finite at iteration %d", k);
            rc = BSM_ENONFINITE;
            break;
        }
        if (o.fixed_iters > 0) {
            if (k == o.fixed_iters) break;
        } else {
            if (r < o.tol) break;
            if (k > 0 && r >= st->r_hist[k - 1]) {
                if (++stall >= 3) {
                    set_error("sign: residual stopped decreasing at %g (iteration %d)", r, k);
                    rc = BSM_ENOCONV;
                    break;
                }
            } else {
                stall = 0;
            }
            if (k == o.max_iter) {
                set_error("sign: no convergence to %g in %d iterations (r = %g)", o.tol, k, r);
                rc = BSM_ENOCONV;
                break;
            }
        }
        rc = multiply(-0.5, *X, *Y, 1.5, *X, o.eps_filter, o.norm, prec, &ms, s);
        st->n_multiplies++;
        st->flops += ms.flops;
        st->n_products += ms.n_products;
        st->smm_ms += ms.smm_ms;
        if (rc != BSM_OK) break;
    }
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
