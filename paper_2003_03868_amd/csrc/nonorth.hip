// Non-orthogonal basis (S != I): S^{1/2}, S^{-1/2} by the coupled
// Newton-Schulz iteration and the density matrix
// P = (I - sign(S^{-1} K - mu I)) S^{-1} / 2 (Sign-Method section, density
// relation), built from the block-sparse multiply, the shift and the sign
// iteration of this library.
//
// Square roots: the second-order sign iteration applied to the block matrix
// [[0, A], [I, 0]] (whose sign is [[0, A^{1/2}], [A^{-1/2}, 0]], the relation
// the Sign-Method section gives for inverses and square roots).  With
// X_k = [[0, Y_k], [Z_k, 0]] the update X (3I - X^2) / 2 acts on the blocks:
//   s = ||S||_inf;  Y_0 = S / s;  Z_0 = I
//   k = 0, 1, ...:  T = filter(Z_k Y_k)      (k = 0: T = Y_0, no product)
//                   r_k = ||T - I||_F / n;  stop if r_k < tol
//                   W = 1.5 I - 0.5 T
//                   Y_{k+1} = filter(Y_k W);  Z_{k+1} = filter(W Z_k)  (k = 0: Z_1 = W)
//   S^{1/2} = sqrt(s) Y;  S^{-1/2} = Z / sqrt(s)
// Three multiplies per iteration (two in the first).
//
// Density: with Z = S^{-1/2}, S^{-1} K - mu I = Z (K~ - mu I) Z^{-1} for the
// symmetric K~ = Z K Z, hence sign(S^{-1} K - mu I) = Z sign(K~ - mu I) Z^{-1}
// and P = Z (I - sign(K~ - mu I)) Z / 2:
//   K~ = filter(filter(Z K) Z);  X = sign(K~ - mu I);  P~ = (I - X) / 2;
//   P = filter(filter(Z P~) Z);  trace(P S) = trace(P~ Z S Z) = trace(P~).
#include <cmath>
#include <cstring>

#include "bsm_internal.h"

namespace bsm {

int sign_iterate(Mat &H, double mu, const bsm_sign_opts &o, Mat **x_out, bsm_sign_stats *st,
                 hipStream_t s);

namespace {

// C = alpha A B (beta = 0), filtered, into a new matrix with A's row and
// B's column block sizes; accumulates the statistics.
int product(double alpha, Mat &A, Mat &B, const bsm_sign_opts &o, Mat **out, bsm_sign_stats *st,
            hipStream_t s) {
    Mat *c = nullptr;
    BSM_TRY(alloc_like_sizes(A, B, &c, s));
    bsm_mult_stats ms{};
    const int rc = multiply(alpha, A, B, 0.0, *c, o.eps_filter, o.norm, BSM_FP64, &ms, s);
    if (rc != BSM_OK) { free_mat(c, s); return rc; }
    st->n_multiplies++;
    st->flops += ms.flops;
    st->n_products += ms.n_products;
    st->smm_launches += ms.smm_launches;
    st->smm_ms += ms.smm_ms;
    *out = c;
    return BSM_OK;
}

// c I with only the diagonal blocks: c (E + I) of the empty matrix E.
int scaled_identity(const Mat &like, double c, Mat **out, hipStream_t s) {
    Mat *e = nullptr;
    BSM_TRY(alloc_like_sizes(like, like, &e, s));
    int rc = dalloc(&e->row_ptr, static_cast<size_t>(e->nbrows) + 1, s);
    if (rc == BSM_OK) {
        hipError_t he = hipMemsetAsync(e->row_ptr, 0, sizeof(int64_t) * (e->nbrows + 1), s);
        if (he != hipSuccess) { set_error("identity: %s", hipGetErrorString(he)); rc = BSM_EDEVICE; }
    }
    if (rc == BSM_OK) rc = compute_blk_off(*e, s);
    if (rc == BSM_OK) rc = shift_scale(*e, -1.0, c, out, s);
    free_mat(e, s);
    return rc;
}

}  // namespace

int sqrt_inv_iterate(Mat &S, const bsm_sign_opts &o, Mat **sqrt_out, Mat **isqrt_out,
                     bsm_sign_stats *st, hipStream_t s) {
    *sqrt_out = nullptr;
    *isqrt_out = nullptr;
    if (S.nbrows != S.nbcols || S.h_rbs != S.h_cbs) {
        set_error("sqrt_inv: S must be square with square diagonal blocks");
        return BSM_EINVAL;
    }
    if (!(o.eps_filter >= 0.0) || !std::isfinite(o.eps_filter) || !(o.tol > 0.0) ||
        o.max_iter < 0 || o.max_iter > 120 ||
        (o.norm != BSM_NORM_FROB && o.norm != BSM_NORM_MAXABS)) {
        set_error("sqrt_inv: need eps_filter >= 0, tol > 0, 0 <= max_iter <= 120, a known norm");
        return BSM_EINVAL;
    }
    hipEvent_t t0, t1;
    BSM_HIP(hipEventCreate(&t0));
    BSM_HIP(hipEventCreate(&t1));
    BSM_HIP(hipEventRecord(t0, s));
    const double n = static_cast<double>(S.nrows);
    double sc = 0.0;
    BSM_TRY(inf_norm(S, 0.0, &sc, s));
    st->scale = sc;
    if (!std::isfinite(sc)) { set_error("sqrt_inv: S holds NaN or Inf"); return BSM_ENONFINITE; }
    if (sc == 0.0) { set_error("sqrt_inv: S is zero"); return BSM_EINVAL; }

    Mat *y = nullptr, *z = nullptr, *t = nullptr, *w = nullptr;
    int rc = shift_scale(S, 0.0, 1.0 / sc, &y, s);
    int stall = 0;
    for (int32_t k = 0; rc == BSM_OK; ++k) {
        if (z) rc = product(1.0, *z, *y, o, &t, st, s);           // T = Z Y
        else rc = shift_scale(*y, 0.0, 1.0, &t, s);               // T_0 = Y_0
        if (rc != BSM_OK) break;
        double d = 0.0;
        rc = sqdist_identity(*t, 1.0, &d, s);
        if (rc != BSM_OK) break;
        const double r = std::sqrt(d) / n;
        st->r_hist[k] = r;
        st->iterations = k;
        if (!std::isfinite(r)) {
            set_error("sqrt_inv: residual is not finite at iteration %d", k);
            rc = BSM_ENONFINITE;
            break;
        }
        if (r < o.tol) break;
        if (k > 0 && r >= st->r_hist[k - 1]) {
            if (++stall >= 3) { set_error("sqrt_inv: residual stalled"); rc = BSM_ENOCONV; break; }
        } else {
            stall = 0;
        }
        if (k >= o.max_iter) { set_error("sqrt_inv: max_iter reached"); rc = BSM_ENOCONV; break; }
        rc = shift_scale(*t, 3.0, -0.5, &w, s);                  // W = 1.5 I - 0.5 T
        free_mat(t, s);
        t = nullptr;
        if (rc != BSM_OK) break;
        Mat *yn = nullptr, *zn = nullptr;
        rc = product(1.0, *y, *w, o, &yn, st, s);                 // Y W
        if (rc == BSM_OK) {
            if (z) {
                rc = product(1.0, *w, *z, o, &zn, st, s);         // W Z
                free_mat(w, s);
            } else {
                zn = w;                                           // Z_1 = W
            }
            w = nullptr;
        }
        if (rc != BSM_OK) { free_mat(yn, s); free_mat(w, s); w = nullptr; break; }
        free_mat(y, s);
        free_mat(z, s);
        y = yn;
        z = zn;
    }
    free_mat(t, s);
    if (rc == BSM_OK || rc == BSM_ENOCONV) {
        Mat *a = nullptr, *b = nullptr;
        int r2 = shift_scale(*y, 0.0, std::sqrt(sc), &a, s);
        if (r2 == BSM_OK) {
            if (z) r2 = shift_scale(*z, 0.0, 1.0 / std::sqrt(sc), &b, s);
            else r2 = scaled_identity(*y, 1.0 / std::sqrt(sc), &b, s);   // stopped with Z_0 = I
        }
        if (r2 == BSM_OK) {
            *sqrt_out = a;
            *isqrt_out = b;
        } else {
            free_mat(a, s);
            rc = r2;
        }
    }
    free_mat(y, s);
    free_mat(z, s);
    (void)hipEventRecord(t1, s);
    (void)hipEventSynchronize(t1);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t0, t1) == hipSuccess) st->device_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return rc;
}

int density_nonorth(Mat &K, Mat &S, double mu, const bsm_sign_opts &o, Mat **p_out,
                    double *trace_ps, bsm_sign_stats *st_sqrt, bsm_sign_stats *st_sign,
                    hipStream_t s) {
    *p_out = nullptr;
    if (K.nbrows != S.nbrows || K.nbcols != S.nbcols || K.h_rbs != S.h_rbs || K.h_cbs != S.h_cbs) {
        set_error("density_nonorth: K and S must have the same block sizes");
        return BSM_EINVAL;
    }
    if (!std::isfinite(mu)) { set_error("density_nonorth: mu must be finite"); return BSM_EINVAL; }
    Mat *sq = nullptr, *z = nullptr, *k1 = nullptr, *kt = nullptr, *x = nullptr, *pt = nullptr,
        *p1 = nullptr;
    int rc = sqrt_inv_iterate(S, o, &sq, &z, st_sqrt, s);
    int first = rc;
    if (rc == BSM_OK || rc == BSM_ENOCONV) rc = product(1.0, *z, K, o, &k1, st_sign, s);
    if (rc == BSM_OK) rc = product(1.0, *k1, *z, o, &kt, st_sign, s);
    if (rc == BSM_OK) {
        bsm_sign_stats ss;
        std::memset(&ss, 0, sizeof(ss));
        rc = sign_iterate(*kt, mu, o, &x, &ss, s);
        // the sign iteration's record, with the transforms' work added
        const int32_t nm = st_sign->n_multiplies;
        const double fl = st_sign->flops;
        const int64_t np = st_sign->n_products;
        const int32_t nl = st_sign->smm_launches;
        const double sm = st_sign->smm_ms;
        *st_sign = ss;
        st_sign->n_multiplies += nm;
        st_sign->flops += fl;
        st_sign->n_products += np;
        st_sign->smm_launches += nl;
        st_sign->smm_ms += sm;
        if (first == BSM_OK) first = rc;
        if (rc != BSM_OK && rc != BSM_ENOCONV) { free_mat(x, s); x = nullptr; }
    }
    if (x && (rc == BSM_OK || rc == BSM_ENOCONV)) {
        int r2 = shift_scale(*x, 1.0, -0.5, &pt, s);            // P~ = (I - X) / 2
        if (r2 == BSM_OK) r2 = trace(*pt, trace_ps, s);
        if (r2 == BSM_OK) r2 = product(1.0, *z, *pt, o, &p1, st_sign, s);
        if (r2 == BSM_OK) r2 = product(1.0, *p1, *z, o, p_out, st_sign, s);
        rc = (r2 == BSM_OK) ? first : r2;
    }
    free_mat(sq, s); free_mat(z, s); free_mat(k1, s); free_mat(kt, s); free_mat(x, s);
    free_mat(pt, s); free_mat(p1, s);
    return rc;
}

}  // namespace bsm
