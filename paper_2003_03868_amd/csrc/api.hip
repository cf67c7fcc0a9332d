// C-ABI entry points of libbsm (declared in include/bsm.h).
#include <algorithm>
#include <cstring>

#include "bsm_internal.h"
#include "plan.h"
#include "smm.h"

namespace bsm {
const char *last_error();
int sign_iterate(Mat &H, double mu, const bsm_sign_opts &o, Mat **x_out, bsm_sign_stats *st,
                 hipStream_t s);
int sqrt_inv_iterate(Mat &S, const bsm_sign_opts &o, Mat **sqrt_out, Mat **isqrt_out,
                     bsm_sign_stats *st, hipStream_t s);
int density_nonorth(Mat &K, Mat &S, double mu, const bsm_sign_opts &o, Mat **p_out,
                    double *trace_ps, bsm_sign_stats *st_sqrt, bsm_sign_stats *st_sign,
                    hipStream_t s);
int trs4_purify(Mat &H, double n_occ, const bsm_sign_opts &o, Mat **p_out, bsm_tc2_stats *st,
                hipStream_t s);
int submatrix_density(Mat &H, double mu, const bsm_sign_opts &o, Mat **p_out, bsm_sub_stats *st,
                      hipStream_t s);
int tc2_purify(Mat &H, double n_occ, const bsm_sign_opts &o, Mat **p_out, bsm_tc2_stats *st,
               hipStream_t s);
}  // namespace bsm

using bsm::Mat;

struct bsm_matrix_s {
    Mat m;
};

struct bsm_plan_s {
    bsm::MulPlan *p = nullptr;
    int *flags = nullptr;        // device record of the executes
    hipStream_t s = nullptr;     // stream of the last call that used the plan: its
                                 // memory is released in that stream's order
};

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static int check_sizes(int32_t n, const int32_t *sz, const char *what) {
    if (n < 0) { bsm::set_error("%s: negative block count", what); return BSM_EINVAL; }
    if (n > 0 && sz == nullptr) { bsm::set_error("%s: block sizes missing", what); return BSM_EINVAL; }
    for (int32_t i = 0; i < n; ++i)
        if (sz[i] < 1 || sz[i] > bsm::kMaxBlock) {
            bsm::set_error("%s: block size %d at %d outside [1, %d]", what, sz[i], i, bsm::kMaxBlock);
            return BSM_EINVAL;
        }
    return BSM_OK;
}

static int upload_sizes(Mat &m, const int32_t *rbs, const int32_t *cbs, hipStream_t s) {
    m.h_rbs.assign(rbs, rbs + m.nbrows);
    m.h_cbs.assign(cbs, cbs + m.nbcols);
    std::vector<int64_t> ro(m.nbrows + 1, 0), co(m.nbcols + 1, 0);
    for (int32_t i = 0; i < m.nbrows; ++i) ro[i + 1] = ro[i] + rbs[i];
    for (int32_t j = 0; j < m.nbcols; ++j) co[j + 1] = co[j] + cbs[j];
    m.nrows = ro[m.nbrows];
    m.ncols = co[m.nbcols];
    m.max_rbs = m.nbrows ? *std::max_element(rbs, rbs + m.nbrows) : 1;
    m.max_cbs = m.nbcols ? *std::max_element(cbs, cbs + m.nbcols) : 1;
    m.uni_r = (m.nbrows && std::all_of(rbs, rbs + m.nbrows, [&](int32_t x) { return x == rbs[0]; })) ? rbs[0] : 0;
    m.uni_c = (m.nbcols && std::all_of(cbs, cbs + m.nbcols, [&](int32_t x) { return x == cbs[0]; })) ? cbs[0] : 0;
    BSM_TRY(bsm::dalloc(&m.rbs, m.nbrows, s));
    BSM_TRY(bsm::dalloc(&m.cbs, m.nbcols, s));
    BSM_TRY(bsm::dalloc(&m.roff, m.nbrows + 1, s));
    BSM_TRY(bsm::dalloc(&m.coff, m.nbcols + 1, s));
    if (m.nbrows) BSM_HIP(hipMemcpyAsync(m.rbs, rbs, sizeof(int32_t) * m.nbrows, hipMemcpyHostToDevice, s));
    if (m.nbcols) BSM_HIP(hipMemcpyAsync(m.cbs, cbs, sizeof(int32_t) * m.nbcols, hipMemcpyHostToDevice, s));
    BSM_HIP(hipMemcpyAsync(m.roff, ro.data(), sizeof(int64_t) * ro.size(), hipMemcpyHostToDevice, s));
    BSM_HIP(hipMemcpyAsync(m.coff, co.data(), sizeof(int64_t) * co.size(), hipMemcpyHostToDevice, s));
    // the host vectors above die at return: make the copies complete first
    BSM_HIP(hipStreamSynchronize(s));
    return BSM_OK;
}

extern "C" {

void bsm_sign_opts_default(bsm_sign_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->eps_filter = 0.0;
    o->tol = 1e-6;
    o->max_iter = 100;
    o->fixed_iters = 0;
    o->norm = BSM_NORM_FROB;
    o->prec = BSM_FP64;
    o->fp64_final_iters = 2;
    o->use_graph = 0;
    o->order = 2;
    o->prec_switch_tol = 1e-4;
}

int bsm_create(bsm_matrix *out, int32_t nbrows, int32_t nbcols, const int32_t *row_blk_size,
               const int32_t *col_blk_size, int64_t nnzb, const int64_t *row_ptr,
               const int32_t *col_idx, const double *values, int on_device, void *stream) {
    bsm::clear_error();
    if (!out) { bsm::set_error("out is NULL"); return BSM_EINVAL; }
    BSM_TRY(check_sizes(nbrows, row_blk_size, "row_blk_size"));
    BSM_TRY(check_sizes(nbcols, col_blk_size, "col_blk_size"));
    if (nnzb < 0 || (nbrows == 0 && nnzb != 0)) { bsm::set_error("bad nnzb"); return BSM_EINVAL; }
    if (row_ptr == nullptr && nbrows > 0) { bsm::set_error("row_ptr is NULL"); return BSM_EINVAL; }
    if (nnzb > 0 && (col_idx == nullptr || values == nullptr)) { bsm::set_error("col_idx/values NULL"); return BSM_EINVAL; }
    hipStream_t s = as_stream(stream);
    auto *h = new bsm_matrix_s;
    Mat &m = h->m;
    int st = hipGetDevice(&m.device) == hipSuccess ? BSM_OK : BSM_EDEVICE;
    m.nbrows = nbrows;
    m.nbcols = nbcols;
    m.nnzb = nnzb;
    m.stream = s;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (st == BSM_OK) st = upload_sizes(m, row_blk_size, col_blk_size, s);
    if (st == BSM_OK) st = bsm::dalloc(&m.row_ptr, nbrows + 1, s);
    if (st == BSM_OK) st = bsm::dalloc(&m.col_idx, nnzb, s);
    if (st == BSM_OK) {
        hipError_t e = hipSuccess;
        if (nbrows > 0) e = hipMemcpyAsync(m.row_ptr, row_ptr, sizeof(int64_t) * (nbrows + 1), kind, s);
        else e = hipMemsetAsync(m.row_ptr, 0, sizeof(int64_t), s);
        if (e == hipSuccess && nnzb > 0) e = hipMemcpyAsync(m.col_idx, col_idx, sizeof(int32_t) * nnzb, kind, s);
        if (e != hipSuccess) { bsm::set_error("create: copy failed: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st == BSM_OK) st = bsm::validate_pattern(m, s);
    if (st == BSM_OK) st = bsm::compute_blk_off(m, s);
    if (st == BSM_OK) {
        int64_t nv = 0;
        hipError_t e = hipMemcpyAsync(&nv, m.blk_off + nnzb, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { bsm::set_error("create: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
        m.nvalues = nv;
    }
    if (st == BSM_OK) st = bsm::dalloc(&m.values, m.nvalues, s);
    if (st == BSM_OK && m.nvalues > 0) {
        hipError_t e = hipMemcpyAsync(m.values, values, sizeof(double) * m.nvalues, kind, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { bsm::set_error("create: values copy failed: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st != BSM_OK) {
        bsm::free_mat_arrays(m, s);
        bsm::dfree(m.rbs, s); bsm::dfree(m.cbs, s); bsm::dfree(m.roff, s); bsm::dfree(m.coff, s);
        delete h;
        return st;
    }
    *out = h;
    return BSM_OK;
}

int bsm_destroy(bsm_matrix h) {
    bsm::clear_error();
    if (!h) return BSM_OK;
    Mat &m = h->m;
    hipStream_t s = m.stream;
    bsm::free_mat_arrays(m, s);
    bsm::dfree(m.rbs, s); bsm::dfree(m.cbs, s); bsm::dfree(m.roff, s); bsm::dfree(m.coff, s);
    delete h;
    return BSM_OK;
}

int bsm_get_info(bsm_matrix h, bsm_info *info) {
    bsm::clear_error();
    if (!h || !info) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    const Mat &m = h->m;
    info->nbrows = m.nbrows; info->nbcols = m.nbcols;
    info->nnzb = m.nnzb; info->nvalues = m.nvalues;
    info->nrows = m.nrows; info->ncols = m.ncols;
    return BSM_OK;
}

int bsm_export(bsm_matrix h, int64_t *row_ptr, int32_t *col_idx, double *values, int on_device,
               void *stream) {
    bsm::clear_error();
    if (!h) { bsm::set_error("NULL handle"); return BSM_EINVAL; }
    Mat &m = h->m;
    hipStream_t s = as_stream(stream);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (row_ptr) BSM_HIP(hipMemcpyAsync(row_ptr, m.row_ptr, sizeof(int64_t) * (m.nbrows + 1), kind, s));
    if (col_idx && m.nnzb) BSM_HIP(hipMemcpyAsync(col_idx, m.col_idx, sizeof(int32_t) * m.nnzb, kind, s));
    if (values && m.nvalues) BSM_HIP(hipMemcpyAsync(values, m.values, sizeof(double) * m.nvalues, kind, s));
    BSM_HIP(hipStreamSynchronize(s));
    return BSM_OK;
}

int bsm_multiply(double alpha, bsm_matrix A, bsm_matrix B, double beta, bsm_matrix C,
                 double eps_filter, int32_t norm, int32_t prec, bsm_mult_stats *stats,
                 void *stream) {
    bsm::clear_error();
    if (!A || !B || !C) { bsm::set_error("NULL handle"); return BSM_EINVAL; }
    if (stats) std::memset(stats, 0, sizeof(*stats));
    return bsm::multiply(alpha, A->m, B->m, beta, C->m, eps_filter, norm, prec, stats,
                         as_stream(stream));
}

int bsm_multiply_plan(double alpha, bsm_matrix A, bsm_matrix B, bsm_matrix C, double eps_filter,
                      int32_t norm, int32_t prec, bsm_plan *plan_out, bsm_mult_stats *stats,
                      void *stream) {
    bsm::clear_error();
    if (!A || !B || !C || !plan_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *plan_out = nullptr;
    if (C == A || C == B) { bsm::set_error("a planned product may not overwrite an operand"); return BSM_EINVAL; }
    if (stats) std::memset(stats, 0, sizeof(*stats));
    hipStream_t s = as_stream(stream);
    bsm::MulPlan *pl = nullptr;
    int st = bsm::multiply(alpha, A->m, B->m, 0.0, C->m, eps_filter, norm, prec, stats, s, &pl);
    if (st != BSM_OK) {
        bsm::free_plan(pl);
        return st;
    }
    bsm_plan_s *h = new bsm_plan_s;
    h->p = pl;
    h->s = s;
    st = bsm::dalloc(&h->flags, 1, s);
    if (st == BSM_OK) st = bsm::zero_flag(h->flags, s);
    if (st != BSM_OK) {
        bsm::dfree(h->flags, s);
        bsm::free_plan(pl);
        delete h;
        return st;
    }
    *plan_out = h;
    return BSM_OK;
}

int bsm_plan_execute(bsm_plan plan, bsm_matrix A, bsm_matrix B, bsm_matrix C, void *stream) {
    bsm::clear_error();
    if (!plan || !A || !B || !C) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    if (C == A || C == B) { bsm::set_error("a planned product may not overwrite an operand"); return BSM_EINVAL; }
    const bsm::MulPlan &p = *plan->p;
    if (C->m.nnzb != p.nnzb || C->m.nvalues != p.nval || C->m.nbrows != A->m.nbrows ||
        C->m.nbcols != B->m.nbcols) {
        bsm::set_error("C does not have the planned product's pattern (%lld blocks, %lld "
                       "scalars expected)", static_cast<long long>(p.nnzb),
                       static_cast<long long>(p.nval));
        return BSM_EINVAL;
    }
    if ((&A->m == &B->m) != p.same_ab) {
        bsm::set_error("the plan was made for %s operands", p.same_ab ? "identical" : "distinct");
        return BSM_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    const int st = bsm::replay_multiply(*plan->p, A->m, B->m, nullptr, C->m.values, plan->flags, s);
    C->m.stream = s;
    plan->s = s;
    plan->p->s = s;
    return st;
}

int bsm_plan_status(bsm_plan plan, int32_t *flags, void *stream) {
    bsm::clear_error();
    if (!plan || !flags) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    hipStream_t s = as_stream(stream);
    int h = 0;
    BSM_HIP(hipMemcpyAsync(&h, plan->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    BSM_HIP(hipStreamSynchronize(s));
    BSM_TRY(bsm::zero_flag(plan->flags, s));
    plan->s = s;
    plan->p->s = s;
    *flags = ((h & bsm::kFlagNonFinite) ? 1 : 0) | ((h & bsm::kFlagPattern) ? 2 : 0);
    return BSM_OK;
}

int bsm_plan_destroy(bsm_plan plan) {
    bsm::clear_error();
    if (!plan) return BSM_OK;
    bsm::dfree(plan->flags, plan->s);
    bsm::free_plan(plan->p);
    delete plan;
    return BSM_OK;
}

int bsm_multiply_screened(double alpha, bsm_matrix A, bsm_matrix B, double beta, bsm_matrix C,
                          double eps_filter, int32_t norm, double eps_screen,
                          bsm_mult_stats *stats, void *stream) {
    bsm::clear_error();
    if (!A || !B || !C) { bsm::set_error("NULL handle"); return BSM_EINVAL; }
    if (!(eps_screen >= 0.0) || !std::isfinite(eps_screen)) {
        bsm::set_error("eps_screen must be finite and >= 0");
        return BSM_EINVAL;
    }
    if (stats) std::memset(stats, 0, sizeof(*stats));
    return bsm::multiply(alpha, A->m, B->m, beta, C->m, eps_filter, norm, BSM_FP64, stats,
                         as_stream(stream), nullptr, eps_screen);
}

int bsm_filter(bsm_matrix h, double eps, int32_t norm, void *stream) {
    bsm::clear_error();
    if (!h) { bsm::set_error("NULL handle"); return BSM_EINVAL; }
    if (!(eps >= 0.0) || !std::isfinite(eps)) { bsm::set_error("eps_filter must be finite and >= 0"); return BSM_EINVAL; }
    if (norm != BSM_NORM_FROB && norm != BSM_NORM_MAXABS) { bsm::set_error("unknown norm"); return BSM_EINVAL; }
    hipStream_t s = as_stream(stream);
    int st = bsm::filter_inplace(h->m, eps, norm, s);
    h->m.stream = s;
    return st;
}

int bsm_block_norms(bsm_matrix h, double *out_dev, void *stream) {
    bsm::clear_error();
    if (!h || (!out_dev && h->m.nnzb)) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    return bsm::block_sqnorms(h->m, out_dev, as_stream(stream));
}

int bsm_trace(bsm_matrix h, double *out, void *stream) {
    bsm::clear_error();
    if (!h || !out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    return bsm::trace(h->m, out, as_stream(stream));
}

int bsm_sqdist_identity(bsm_matrix h, double shift, double *out, void *stream) {
    bsm::clear_error();
    if (!h || !out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    return bsm::sqdist_identity(h->m, shift, out, as_stream(stream));
}

int bsm_sqdist_identity_noalloc(bsm_matrix h, double shift, double *out_dev, void *stream) {
    bsm::clear_error();
    if (!h || !out_dev) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    return bsm::sqdist_identity_noalloc(h->m, shift, out_dev, as_stream(stream));
}

int bsm_inf_norm(bsm_matrix h, double mu, double *out, void *stream) {
    bsm::clear_error();
    if (!h || !out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    return bsm::inf_norm(h->m, mu, out, as_stream(stream));
}

int bsm_shift_scale(bsm_matrix A, double mu, double scale, bsm_matrix *out, void *stream) {
    bsm::clear_error();
    if (!A || !out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    Mat *m = nullptr;
    BSM_TRY(bsm::shift_scale(A->m, mu, scale, &m, as_stream(stream)));
    auto *h = new bsm_matrix_s;
    h->m = std::move(*m);
    delete m;
    *out = h;
    return BSM_OK;
}

int bsm_add(double alpha, bsm_matrix A, double beta, bsm_matrix B, double gamma,
            double eps_filter, int32_t norm, bsm_matrix *out, void *stream) {
    bsm::clear_error();
    if (!A || !out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    Mat *m = nullptr;
    BSM_TRY(bsm::add_mat(alpha, A->m, beta, B ? &B->m : nullptr, gamma, eps_filter, norm, &m,
                         as_stream(stream)));
    auto *h = new bsm_matrix_s;
    h->m = std::move(*m);
    delete m;
    *out = h;
    return BSM_OK;
}

int bsm_sign_iterate(bsm_matrix H, double mu, const bsm_sign_opts *opts, bsm_matrix *x_out,
                     bsm_sign_stats *stats, void *stream) {
    bsm::clear_error();
    if (!H || !x_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    bsm_sign_opts o;
    if (opts) o = *opts; else bsm_sign_opts_default(&o);
    bsm_sign_stats local;
    bsm_sign_stats *st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    Mat *x = nullptr;
    int rc = bsm::sign_iterate(H->m, mu, o, &x, st, as_stream(stream));
    if (x) {
        auto *h = new bsm_matrix_s;
        h->m = std::move(*x);
        delete x;
        *x_out = h;
    }
    return rc;
}

int bsm_mu_bisect(bsm_matrix H, double n_target, double mu_lo, double mu_hi, double count_tol,
                  int32_t max_steps, const bsm_sign_opts *opts, double *mu_out,
                  bsm_matrix *x_out, bsm_mu_stats *stats, void *stream) {
    bsm::clear_error();
    if (!H || !x_out || !mu_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *x_out = nullptr;
    if (!std::isfinite(mu_lo) || !std::isfinite(mu_hi) || !(mu_lo < mu_hi) ||
        !std::isfinite(n_target) || !(count_tol > 0.0) || !std::isfinite(count_tol) ||
        max_steps < 1 || max_steps > 64) {
        bsm::set_error("mu_bisect: need finite mu_lo < mu_hi, finite n_target, count_tol > 0 "
                       "and 1 <= max_steps <= 64");
        return BSM_EINVAL;
    }
    bsm_sign_opts o;
    if (opts) o = *opts; else bsm_sign_opts_default(&o);
    bsm_mu_stats local;
    bsm_mu_stats *ms = stats ? stats : &local;
    std::memset(ms, 0, sizeof(*ms));
    hipStream_t s = as_stream(stream);
    double lo = mu_lo, hi = mu_hi;
    Mat *x = nullptr;
    int rc = BSM_ENOCONV;
    double mu = 0.0;
    for (int32_t t = 0; t < max_steps; ++t) {
        mu = 0.5 * (lo + hi);
        if (x) { bsm::free_mat(x, s); x = nullptr; }
        bsm_sign_stats st;
        std::memset(&st, 0, sizeof(st));
        const int src = bsm::sign_iterate(H->m, mu, o, &x, &st, s);
        ms->flops += st.flops;
        ms->device_ms += st.device_ms;
        if (src != BSM_OK && src != BSM_ENOCONV) {
            if (x) bsm::free_mat(x, s);
            return src;
        }
        if (src == BSM_ENOCONV) ms->sign_noconv++;
        const double count = st.trace_p;
        ms->mu_hist[t] = mu;
        ms->count_hist[t] = count;
        ms->steps = t + 1;
        if (std::fabs(count - n_target) <= count_tol) { rc = BSM_OK; break; }
        if (count < n_target) lo = mu; else hi = mu;
    }
    if (rc == BSM_ENOCONV)
        bsm::set_error("mu_bisect: count not within count_tol after %d steps", max_steps);
    *mu_out = mu;
    if (x) {
        auto *h = new bsm_matrix_s;
        h->m = std::move(*x);
        delete x;
        *x_out = h;
    }
    return rc;
}

static bsm_matrix wrap(Mat *m) {
    auto *h = new bsm_matrix_s;
    h->m = std::move(*m);
    delete m;
    return h;
}

int bsm_sqrt_inv(bsm_matrix S, const bsm_sign_opts *opts, bsm_matrix *sqrt_out,
                 bsm_matrix *isqrt_out, bsm_sign_stats *stats, void *stream) {
    bsm::clear_error();
    if (!S || !sqrt_out || !isqrt_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *sqrt_out = nullptr;
    *isqrt_out = nullptr;
    bsm_sign_opts o;
    if (opts) o = *opts; else bsm_sign_opts_default(&o);
    bsm_sign_stats local;
    bsm_sign_stats *st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    Mat *a = nullptr, *b = nullptr;
    const int rc = bsm::sqrt_inv_iterate(S->m, o, &a, &b, st, as_stream(stream));
    if (a) *sqrt_out = wrap(a);
    if (b) *isqrt_out = wrap(b);
    return rc;
}

int bsm_density_nonorth(bsm_matrix K, bsm_matrix S, double mu, const bsm_sign_opts *opts,
                        bsm_matrix *p_out, double *trace_ps, bsm_sign_stats *sqrt_stats,
                        bsm_sign_stats *sign_stats, void *stream) {
    bsm::clear_error();
    if (!K || !S || !p_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *p_out = nullptr;
    bsm_sign_opts o;
    if (opts) o = *opts; else bsm_sign_opts_default(&o);
    bsm_sign_stats l1, l2;
    bsm_sign_stats *s1 = sqrt_stats ? sqrt_stats : &l1;
    bsm_sign_stats *s2 = sign_stats ? sign_stats : &l2;
    std::memset(s1, 0, sizeof(*s1));
    std::memset(s2, 0, sizeof(*s2));
    double tps = 0.0;
    Mat *p = nullptr;
    const int rc = bsm::density_nonorth(K->m, S->m, mu, o, &p, &tps, s1, s2, as_stream(stream));
    if (trace_ps) *trace_ps = tps;
    if (p) *p_out = wrap(p);
    return rc;
}

int bsm_tc2(bsm_matrix H, double n_occ, const bsm_sign_opts *opts, bsm_matrix *p_out,
            bsm_tc2_stats *stats, void *stream) {
    bsm::clear_error();
    if (!H || !p_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *p_out = nullptr;
    bsm_sign_opts o;
    if (opts) o = *opts; else bsm_sign_opts_default(&o);
    bsm_tc2_stats local;
    bsm_tc2_stats *st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    Mat *p = nullptr;
    const int rc = bsm::tc2_purify(H->m, n_occ, o, &p, st, as_stream(stream));
    if (p) *p_out = wrap(p);
    return rc;
}

int bsm_trs4(bsm_matrix H, double n_occ, const bsm_sign_opts *opts, bsm_matrix *p_out,
             bsm_tc2_stats *stats, void *stream) {
    bsm::clear_error();
    if (!H || !p_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *p_out = nullptr;
    bsm_sign_opts o;
    if (opts) o = *opts; else bsm_sign_opts_default(&o);
    bsm_tc2_stats local;
    bsm_tc2_stats *st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    Mat *p = nullptr;
    const int rc = bsm::trs4_purify(H->m, n_occ, o, &p, st, as_stream(stream));
    if (p) *p_out = wrap(p);
    return rc;
}

int bsm_submatrix_density(bsm_matrix H, double mu, const bsm_sign_opts *opts, bsm_matrix *p_out,
                          bsm_sub_stats *stats, void *stream) {
    bsm::clear_error();
    if (!H || !p_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *p_out = nullptr;
    bsm_sign_opts o;
    if (opts) o = *opts; else bsm_sign_opts_default(&o);
    bsm_sub_stats local;
    bsm_sub_stats *st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    Mat *p = nullptr;
    const int rc = bsm::submatrix_density(H->m, mu, o, &p, st, as_stream(stream));
    if (p) *p_out = wrap(p);
    return rc;
}

int bsm_transpose(bsm_matrix A, bsm_matrix *out, void *stream) {
    bsm::clear_error();
    if (!A || !out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    *out = nullptr;
    Mat *m = nullptr;
    BSM_TRY(bsm::transpose_mat(A->m, &m, as_stream(stream)));
    *out = wrap(m);
    return BSM_OK;
}

int bsm_density_from_sign(bsm_matrix X, bsm_matrix *p_out, double *trace_p, void *stream) {
    bsm::clear_error();
    if (!X || !p_out) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    hipStream_t s = as_stream(stream);
    Mat *m = nullptr;
    BSM_TRY(bsm::shift_scale(X->m, 1.0, -0.5, &m, s));
    if (trace_p) {
        int st = bsm::trace(*m, trace_p, s);
        if (st != BSM_OK) { bsm::free_mat(m, s); return st; }
    }
    auto *h = new bsm_matrix_s;
    h->m = std::move(*m);
    delete m;
    *p_out = h;
    return BSM_OK;
}

int bsm_smm_bench(int32_t m, int32_t n, int32_t k, int64_t n_cblocks, int32_t prods_per_cblock,
                  int32_t n_params, const bsm_smm_params *params, int32_t reps, double *ms_out,
                  void *stream) {
    bsm::clear_error();
    if (!params || !ms_out || n_params < 1) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    static_assert(sizeof(bsm_smm_params) == sizeof(bsm::SmmParams), "params layout");
    return bsm::smm_bench(m, n, k, n_cblocks, prods_per_cblock, n_params,
                          reinterpret_cast<const bsm::SmmParams *>(params), reps, ms_out,
                          as_stream(stream));
}

int bsm_set_smm_table(int32_t n_entries, const int32_t *mnk, const bsm_smm_params *params) {
    bsm::clear_error();
    if (n_entries > 0 && (!mnk || !params)) { bsm::set_error("NULL argument"); return BSM_EINVAL; }
    for (int32_t i = 0; i < n_entries; ++i) {
        const bsm_smm_params &p = params[i];
        if (p.family < 0 || p.family > 3 || (p.wpg != 1 && p.wpg != 2 && p.wpg != 4) ||
            (p.prefetch != 0 && p.prefetch != 1)) {
            bsm::set_error("bad parameters in entry %d", i);
            return BSM_EINVAL;
        }
        if (mnk[3 * i] < 1 || mnk[3 * i] > bsm::kMaxBlock || mnk[3 * i + 1] < 1 ||
            mnk[3 * i + 1] > bsm::kMaxBlock || mnk[3 * i + 2] < 0 || mnk[3 * i + 2] > bsm::kMaxBlock) {
            bsm::set_error("bad (m, n, k) in entry %d", i);
            return BSM_EINVAL;
        }
    }
    bsm::table_set(n_entries, mnk, reinterpret_cast<const bsm::SmmParams *>(params));
    return BSM_OK;
}

const char *bsm_last_error(void) { return bsm::last_error(); }

const char *bsm_version(void) { return "bsm 0.1 (gfx950)"; }

const char *bsm_last_smm_kernel(void) { return bsm::last_kernel(); }

}  // extern "C"
