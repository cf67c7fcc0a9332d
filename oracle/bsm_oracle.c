/*
 * CPU oracle for the block-sparse multiply, the norm filter and the
 * Newton-Schulz sign iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP library against a plain,
 * slow, obviously correct reference.  It shares no code, header or helper
 * with the HIP library.
 *
 * Everything here is plain C, FP64, explicit loops, no BLAS, compiled with
 * -O3 -ffp-contract=off so that no multiply-add is fused.  OpenMP only
 * splits independent block rows between threads; each output element is
 * summed by one thread in ascending k.
 *
 * Matrix layout (the blocked CSR of the DBCSR section): block-row pointers
 * row_ptr[nbrows+1] (int64), column indices col_idx[nnzb] (int32, strictly
 * increasing per row), values = stored blocks concatenated in CSR order, each
 * block row-major, of size row_blk_size[i] x col_blk_size[j].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nbrows, nbcols;
    const int32_t *rbs;   /* row block sizes  [nbrows] */
    const int32_t *cbs;   /* col block sizes  [nbcols] */
    int64_t nnzb;
    int64_t *row_ptr;     /* [nbrows+1] */
    int32_t *col_idx;     /* [nnzb] */
    double *values;       /* concatenated row-major blocks */
} omat;

enum { ORC_NORM_FROB = 0, ORC_NORM_MAXABS = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENOCONV = -4,
       ORC_ENONFINITE = -5 };

/* ---------------------------------------------------------------- helpers */

static int64_t *block_offsets(const omat *a)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(a->nnzb + 1));
    if (!off) return NULL;
    off[0] = 0;
    for (int32_t i = 0; i < a->nbrows; ++i)
        for (int64_t t = a->row_ptr[i]; t < a->row_ptr[i + 1]; ++t)
            off[t + 1] = off[t] + (int64_t)a->rbs[i] * a->cbs[a->col_idx[t]];
    return off;
}

/* Position of block (i, j) in a, or -1 (binary search in row i). */
static int64_t find_block(const omat *a, int32_t i, int32_t j)
{
    int64_t lo = a->row_ptr[i], hi = a->row_ptr[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a->col_idx[mid] == j) return mid;
        if (a->col_idx[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

void orc_free(omat *m)
{
    if (!m) return;
    free(m->row_ptr); free(m->col_idx); free(m->values);
    m->row_ptr = NULL; m->col_idx = NULL; m->values = NULL; m->nnzb = 0;
}

/*
 * Keep test of the norm filter (Sign-Method section: after every product,
 * entries below eps_filter are flushed to zero to retain sparsity).  Read at
 * block granularity: FROB drops a block iff sum(x^2) < eps^2, MAXABS drops it
 * iff max|x| < eps.  With eps = 0 nothing is dropped.
 */
static int keep_block(const double *x, int64_t len, double eps, int kind)
{
    if (kind == ORC_NORM_MAXABS) {
        double mx = 0.0;
        for (int64_t e = 0; e < len; ++e) { double v = fabs(x[e]); if (v > mx) mx = v; }
        return !(mx < eps);
    }
    double s = 0.0;
    for (int64_t e = 0; e < len; ++e) s += x[e] * x[e];
    return !(s < eps * eps);
}

/* Squared Frobenius norm of every stored block, in storage order. */
int orc_block_sqnorms(const omat *a, double *out)
{
    int64_t *off = block_offsets(a);
    if (!off) return ORC_ENOMEM;
    for (int64_t t = 0; t < a->nnzb; ++t) {
        double s = 0.0;
        for (int64_t e = off[t]; e < off[t + 1]; ++e) s += a->values[e] * a->values[e];
        out[t] = s;
    }
    free(off);
    return ORC_OK;
}

/* ----------------------------------------------------- per-row assembly */

typedef struct {
    int64_t nblk, cap_blk, nval, cap_val;
    int32_t *cols;
    double *vals;
} rowbuf;

static int rowbuf_push(rowbuf *r, int32_t j, const double *blk, int64_t len)
{
    if (r->nblk == r->cap_blk) {
        int64_t c = r->cap_blk ? 2 * r->cap_blk : 16;
        int32_t *p = (int32_t *)realloc(r->cols, sizeof(int32_t) * (size_t)c);
        if (!p) return ORC_ENOMEM;
        r->cols = p; r->cap_blk = c;
    }
    if (r->nval + len > r->cap_val) {
        int64_t c = r->cap_val ? 2 * r->cap_val : 1024;
        while (c < r->nval + len) c *= 2;
        double *p = (double *)realloc(r->vals, sizeof(double) * (size_t)c);
        if (!p) return ORC_ENOMEM;
        r->vals = p; r->cap_val = c;
    }
    r->cols[r->nblk++] = j;
    memcpy(r->vals + r->nval, blk, sizeof(double) * (size_t)len);
    r->nval += len;
    return ORC_OK;
}

static int assemble(omat *out, int32_t nbrows, int32_t nbcols, const int32_t *rbs,
                    const int32_t *cbs, rowbuf *rows)
{
    int64_t nnzb = 0, nval = 0;
    for (int32_t i = 0; i < nbrows; ++i) { nnzb += rows[i].nblk; nval += rows[i].nval; }
    out->nbrows = nbrows; out->nbcols = nbcols; out->rbs = rbs; out->cbs = cbs;
    out->nnzb = nnzb;
    out->row_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nbrows + 1));
    out->col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnzb ? nnzb : 1));
    out->values = (double *)malloc(sizeof(double) * (size_t)(nval ? nval : 1));
    if (!out->row_ptr || !out->col_idx || !out->values) { orc_free(out); return ORC_ENOMEM; }
    int64_t pb = 0, pv = 0;
    out->row_ptr[0] = 0;
    for (int32_t i = 0; i < nbrows; ++i) {
        if (rows[i].nblk) memcpy(out->col_idx + pb, rows[i].cols, sizeof(int32_t) * (size_t)rows[i].nblk);
        if (rows[i].nval) memcpy(out->values + pv, rows[i].vals, sizeof(double) * (size_t)rows[i].nval);
        pb += rows[i].nblk; pv += rows[i].nval;
        out->row_ptr[i + 1] = pb;
    }
    return ORC_OK;
}

static void free_rows(rowbuf *rows, int32_t n)
{
    for (int32_t i = 0; i < n; ++i) { free(rows[i].cols); free(rows[i].vals); }
    free(rows);
}

/* ------------------------------------------------------------- multiply */

/*
 * C = alpha * A * B + beta * Cin, then the norm filter.  This is the plain
 * definition behind the DBCSR multiply (DBCSR section: matrix multiplication
 * of blocked-CSR matrices; local multiplication as pairwise products of small
 * dense blocks, C = C + A*B):
 *
 *   stored pattern S = {(i,j) : some k has A_ik and B_kj stored}
 *                      union pattern(Cin) when beta != 0;
 *   C_ij = alpha * sum_k A_ik B_kj + beta * Cin_ij  for (i,j) in S;
 *   keep block (i,j) iff it passes the filter.
 *
 * Each C_ij is summed over k ascending, and inside a block product over the
 * inner index ascending.  cin may be NULL (treated as empty); with beta == 0
 * its pattern and values are ignored.
 *
 * Product-level norm screening (the screening of the Sign-Method section's
 * discussion of sparsity; tau > 0): the term A_ik B_kj is left out of the
 * sum when ||A_ik||_F^2 ||B_kj||_F^2 < tau^2 (squared Frobenius norms in
 * FP64, summed in storage order).  The stored pattern is that of the
 * unscreened product; a block whose terms were all left out holds
 * beta C_in (or zeros) before the filter.  tau = 0 screens nothing.
 */
static double block_sq(const double *x, int64_t len)
{
    double s = 0.0;
    for (int64_t t = 0; t < len; ++t) s += x[t] * x[t];
    return s;
}

int orc_multiply_screened(double alpha, const omat *a, const omat *b, double beta,
                          const omat *cin, double eps, int norm_kind, double tau, omat *out)
{
    if (a->nbcols != b->nbrows) return ORC_EINVAL;
    for (int32_t k = 0; k < a->nbcols; ++k) if (a->cbs[k] != b->rbs[k]) return ORC_EINVAL;
    for (int32_t i = 0; i < a->nbrows; ++i) if (a->rbs[i] < 1 || a->rbs[i] > 64) return ORC_EINVAL;
    for (int32_t j = 0; j < b->nbcols; ++j) if (b->cbs[j] < 1 || b->cbs[j] > 64) return ORC_EINVAL;
    if (eps < 0 || !(tau >= 0.0)) return ORC_EINVAL;
    const double tau2 = tau * tau;
    int use_c = (beta != 0.0) && cin != NULL;
    if (use_c && (cin->nbrows != a->nbrows || cin->nbcols != b->nbcols)) return ORC_EINVAL;

    int64_t *aoff = block_offsets(a), *boff = block_offsets(b);
    int64_t *coff = use_c ? block_offsets(cin) : NULL;
    rowbuf *rows = (rowbuf *)calloc((size_t)(a->nbrows ? a->nbrows : 1), sizeof(rowbuf));
    if (!aoff || !boff || (use_c && !coff) || !rows) {
        free(aoff); free(boff); free(coff); free(rows); return ORC_ENOMEM;
    }
    int status = ORC_OK;

#pragma omp parallel
    {
        unsigned char *mark = (unsigned char *)calloc((size_t)(b->nbcols ? b->nbcols : 1), 1);
        double *acc = (double *)malloc(sizeof(double) * 64 * 64);
        if (!mark || !acc) {
#pragma omp atomic write
            status = ORC_ENOMEM;
        }
#pragma omp for schedule(static)
        for (int32_t i = 0; i < a->nbrows; ++i) {
            if (!mark || !acc) continue;
            const int32_t m = a->rbs[i];
            /* pattern of row i */
            for (int64_t ta = a->row_ptr[i]; ta < a->row_ptr[i + 1]; ++ta) {
                int32_t k = a->col_idx[ta];
                for (int64_t tb = b->row_ptr[k]; tb < b->row_ptr[k + 1]; ++tb)
                    mark[b->col_idx[tb]] = 1;
            }
            if (use_c)
                for (int64_t tc = cin->row_ptr[i]; tc < cin->row_ptr[i + 1]; ++tc)
                    mark[cin->col_idx[tc]] = 1;
            for (int32_t j = 0; j < b->nbcols; ++j) {
                if (!mark[j]) continue;
                mark[j] = 0;
                const int32_t n = b->cbs[j];
                for (int e = 0; e < m * n; ++e) acc[e] = 0.0;
                for (int64_t ta = a->row_ptr[i]; ta < a->row_ptr[i + 1]; ++ta) {
                    int32_t k = a->col_idx[ta];
                    int64_t tb = find_block(b, k, j);
                    if (tb < 0) continue;
                    const int32_t kk = a->cbs[k];
                    const double *ab = a->values + aoff[ta];
                    const double *bb = b->values + boff[tb];
                    if (tau > 0.0 && block_sq(ab, (int64_t)m * kk) * block_sq(bb, (int64_t)kk * n) < tau2)
                        continue;                       /* screened term */
                    for (int r = 0; r < m; ++r)
                        for (int t = 0; t < kk; ++t) {
                            const double av = ab[r * kk + t];
                            for (int c = 0; c < n; ++c)
                                acc[r * n + c] += av * bb[t * n + c];
                        }
                }
                for (int e = 0; e < m * n; ++e) acc[e] *= alpha;
                if (use_c) {
                    int64_t tc = find_block(cin, i, j);
                    if (tc >= 0) {
                        const double *cb = cin->values + coff[tc];
                        for (int e = 0; e < m * n; ++e) acc[e] += beta * cb[e];
                    }
                }
                if (keep_block(acc, (int64_t)m * n, eps, norm_kind))
                    if (rowbuf_push(&rows[i], j, acc, (int64_t)m * n) != ORC_OK) {
#pragma omp atomic write
                        status = ORC_ENOMEM;
                    }
            }
        }
        free(mark); free(acc);
    }
    if (status == ORC_OK)
        status = assemble(out, a->nbrows, b->nbcols, a->rbs, b->cbs, rows);
    free_rows(rows, a->nbrows);
    free(aoff); free(boff); free(coff);
    return status;
}

/* The unscreened multiply. */
int orc_multiply(double alpha, const omat *a, const omat *b, double beta,
                 const omat *cin, double eps, int norm_kind, omat *out)
{
    return orc_multiply_screened(alpha, a, b, beta, cin, eps, norm_kind, 0.0, out);
}

/* Filter a matrix on its own (same keep test as after a multiply). */
int orc_filter(const omat *a, double eps, int norm_kind, omat *out)
{
    if (eps < 0) return ORC_EINVAL;
    int64_t *off = block_offsets(a);
    rowbuf *rows = (rowbuf *)calloc((size_t)(a->nbrows ? a->nbrows : 1), sizeof(rowbuf));
    if (!off || !rows) { free(off); free(rows); return ORC_ENOMEM; }
    int status = ORC_OK;
    for (int32_t i = 0; i < a->nbrows && status == ORC_OK; ++i)
        for (int64_t t = a->row_ptr[i]; t < a->row_ptr[i + 1]; ++t) {
            int64_t len = off[t + 1] - off[t];
            if (keep_block(a->values + off[t], len, eps, norm_kind))
                status = rowbuf_push(&rows[i], a->col_idx[t], a->values + off[t], len);
        }
    if (status == ORC_OK)
        status = assemble(out, a->nbrows, a->nbcols, a->rbs, a->cbs, rows);
    free_rows(rows, a->nbrows);
    free(off);
    return status;
}

/* --------------------------------------------------- whole-matrix scalars */

/* trace(A) for a square block matrix (DBCSR single-matrix operation). */
double orc_trace(const omat *a)
{
    int64_t *off = block_offsets(a);
    double tr = 0.0;
    for (int32_t i = 0; i < a->nbrows; ++i) {
        int64_t t = find_block(a, i, i);
        if (t < 0) continue;
        const int32_t m = a->rbs[i];
        for (int r = 0; r < m; ++r) tr += a->values[off[t] + (int64_t)r * m + r];
    }
    free(off);
    return tr;
}

/* ||A - shift*I||_F^2 with missing diagonal blocks counted as -shift*I. */
double orc_sqdist_identity(const omat *a, double shift)
{
    int64_t *off = block_offsets(a);
    double s = 0.0;
    for (int32_t i = 0; i < a->nbrows; ++i) {
        const int32_t m = a->rbs[i];
        int have_diag = 0;
        for (int64_t t = a->row_ptr[i]; t < a->row_ptr[i + 1]; ++t) {
            const int32_t j = a->col_idx[t];
            const int32_t n = a->cbs[j];
            const double *x = a->values + off[t];
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < n; ++c) {
                    double v = x[r * n + c] - ((j == i && r == c) ? shift : 0.0);
                    s += v * v;
                }
            if (j == i) have_diag = 1;
        }
        if (!have_diag) s += (double)m * shift * shift;
    }
    free(off);
    return s;
}

/* max over scalar rows of sum |a_rc| of (A - mu*I): the infinity norm. */
double orc_inf_norm_shifted(const omat *a, double mu)
{
    int64_t *off = block_offsets(a);
    double best = 0.0;
    for (int32_t i = 0; i < a->nbrows; ++i) {
        const int32_t m = a->rbs[i];
        for (int r = 0; r < m; ++r) {
            double s = 0.0;
            int have_diag = 0;
            for (int64_t t = a->row_ptr[i]; t < a->row_ptr[i + 1]; ++t) {
                const int32_t j = a->col_idx[t];
                const int32_t n = a->cbs[j];
                const double *x = a->values + off[t] + (int64_t)r * n;
                for (int c = 0; c < n; ++c)
                    s += fabs(x[c] - ((j == i && c == r) ? mu : 0.0));
                if (j == i) have_diag = 1;
            }
            if (!have_diag) s += fabs(mu);
            if (s > best) best = s;
        }
    }
    free(off);
    return best;
}

/*
 * out = scale * (A - mu*I), inserting a diagonal block where one is missing
 * (needed for the shifted start X_0 of the sign iteration).
 */
int orc_shift_scale(const omat *a, double mu, double scale, omat *out)
{
    for (int32_t i = 0; i < a->nbrows; ++i) if (a->rbs[i] < 1 || a->rbs[i] > 64) return ORC_EINVAL;
    for (int32_t j = 0; j < a->nbcols; ++j) if (a->cbs[j] < 1 || a->cbs[j] > 64) return ORC_EINVAL;
    int64_t *off = block_offsets(a);
    rowbuf *rows = (rowbuf *)calloc((size_t)(a->nbrows ? a->nbrows : 1), sizeof(rowbuf));
    double *tmp = (double *)malloc(sizeof(double) * 64 * 64);
    if (!off || !rows || !tmp) { free(off); free(rows); free(tmp); return ORC_ENOMEM; }
    int status = ORC_OK;
    for (int32_t i = 0; i < a->nbrows && status == ORC_OK; ++i) {
        const int32_t m = a->rbs[i];
        int64_t t = a->row_ptr[i];
        int done_diag = 0;
        for (;;) {
            int32_t j = (t < a->row_ptr[i + 1]) ? a->col_idx[t] : a->nbcols;
            if (!done_diag && j > i) {          /* missing diagonal block */
                for (int e = 0; e < m * m; ++e) tmp[e] = 0.0;
                for (int r = 0; r < m; ++r) tmp[r * m + r] = -scale * mu;
                status = rowbuf_push(&rows[i], i, tmp, (int64_t)m * m);
                done_diag = 1;
                if (status != ORC_OK) break;
            }
            if (t >= a->row_ptr[i + 1]) break;
            const int32_t n = a->cbs[j];
            for (int e = 0; e < m * n; ++e) tmp[e] = scale * a->values[off[t] + e];
            if (j == i) {
                for (int r = 0; r < m; ++r) tmp[r * m + r] = scale * (a->values[off[t] + (int64_t)r * m + r] - mu);
                done_diag = 1;
            }
            status = rowbuf_push(&rows[i], j, tmp, (int64_t)m * n);
            if (status != ORC_OK) break;
            ++t;
        }
    }
    if (status == ORC_OK)
        status = assemble(out, a->nbrows, a->nbcols, a->rbs, a->cbs, rows);
    free_rows(rows, a->nbrows);
    free(off); free(tmp);
    return status;
}

/*
 * B = A^T, the transpose among the DBCSR library's operations: block (i, j)
 * of A (m x n, row-major) becomes block (j, i) of B, its n x m transpose.
 * Rows of A are walked in ascending order, so every row of B receives its
 * columns in ascending order.
 */
int orc_transpose(const omat *a, omat *out)
{
    for (int32_t i = 0; i < a->nbrows; ++i) if (a->rbs[i] < 1 || a->rbs[i] > 64) return ORC_EINVAL;
    for (int32_t j = 0; j < a->nbcols; ++j) if (a->cbs[j] < 1 || a->cbs[j] > 64) return ORC_EINVAL;
    int64_t *off = block_offsets(a);
    rowbuf *rows = (rowbuf *)calloc((size_t)(a->nbcols ? a->nbcols : 1), sizeof(rowbuf));
    double *tmp = (double *)malloc(sizeof(double) * 64 * 64);
    if (!off || !rows || !tmp) { free(off); free(rows); free(tmp); return ORC_ENOMEM; }
    int status = ORC_OK;
    for (int32_t i = 0; i < a->nbrows && status == ORC_OK; ++i) {
        const int32_t m = a->rbs[i];
        for (int64_t t = a->row_ptr[i]; t < a->row_ptr[i + 1] && status == ORC_OK; ++t) {
            const int32_t j = a->col_idx[t];
            const int32_t n = a->cbs[j];
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < n; ++c) tmp[c * m + r] = a->values[off[t] + (int64_t)r * n + c];
            status = rowbuf_push(&rows[j], i, tmp, (int64_t)m * n);
        }
    }
    if (status == ORC_OK)
        status = assemble(out, a->nbcols, a->nbrows, a->cbs, a->rbs, rows);
    free_rows(rows, a->nbcols);
    free(off); free(tmp);
    return status;
}

/*
 * C = alpha * A + beta * B + gamma * I, then the norm filter: the matrix sum
 * of the DBCSR operations (DBCSR section lists multiply, sum, trace and
 * transpose).  Stored pattern = pattern(A) union pattern(B), plus the diagonal
 * blocks when gamma != 0 (square diagonal blocks required then).  Per element
 * v = alpha*a + beta*b with a, b = 0 where a block is absent, then v += gamma
 * on the diagonal.  b may be NULL (empty).
 */
int orc_add(double alpha, const omat *a, double beta, const omat *b, double gamma,
            double eps, int norm_kind, omat *out)
{
    if (b && (a->nbrows != b->nbrows || a->nbcols != b->nbcols)) return ORC_EINVAL;
    for (int32_t i = 0; i < a->nbrows; ++i) if (a->rbs[i] < 1 || a->rbs[i] > 64) return ORC_EINVAL;
    for (int32_t j = 0; j < a->nbcols; ++j) if (a->cbs[j] < 1 || a->cbs[j] > 64) return ORC_EINVAL;
    if (b) {
        for (int32_t i = 0; i < a->nbrows; ++i) if (a->rbs[i] != b->rbs[i]) return ORC_EINVAL;
        for (int32_t j = 0; j < a->nbcols; ++j) if (a->cbs[j] != b->cbs[j]) return ORC_EINVAL;
    }
    if (gamma != 0.0) {
        if (a->nbrows != a->nbcols) return ORC_EINVAL;
        for (int32_t i = 0; i < a->nbrows; ++i) if (a->rbs[i] != a->cbs[i]) return ORC_EINVAL;
    }
    if (eps < 0) return ORC_EINVAL;
    int64_t *offa = block_offsets(a);
    int64_t *offb = b ? block_offsets(b) : NULL;
    rowbuf *rows = (rowbuf *)calloc((size_t)(a->nbrows ? a->nbrows : 1), sizeof(rowbuf));
    double *tmp = (double *)malloc(sizeof(double) * 64 * 64);
    if (!offa || (b && !offb) || !rows || !tmp) {
        free(offa); free(offb); free(rows); free(tmp);
        return ORC_ENOMEM;
    }
    int status = ORC_OK;
    for (int32_t i = 0; i < a->nbrows && status == ORC_OK; ++i) {
        const int32_t m = a->rbs[i];
        int64_t ta = a->row_ptr[i], tb = b ? b->row_ptr[i] : 0;
        const int64_t ea = a->row_ptr[i + 1], eb = b ? b->row_ptr[i + 1] : 0;
        int done_diag = (gamma == 0.0);
        for (;;) {
            const int32_t ja = ta < ea ? a->col_idx[ta] : a->nbcols;
            const int32_t jb = tb < eb ? b->col_idx[tb] : a->nbcols;
            const int32_t jd = done_diag ? a->nbcols : i;
            int32_t j = ja < jb ? ja : jb;
            if (jd < j) j = jd;
            if (j >= a->nbcols) break;
            if (j == i) done_diag = 1;
            const int32_t n = a->cbs[j];
            for (int e = 0; e < m * n; ++e) tmp[e] = 0.0;
            if (ja == j) {
                for (int e = 0; e < m * n; ++e) tmp[e] = alpha * a->values[offa[ta] + e];
                ++ta;
            }
            if (jb == j) {
                for (int e = 0; e < m * n; ++e) tmp[e] = tmp[e] + beta * b->values[offb[tb] + e];
                ++tb;
            }
            if (j == i && gamma != 0.0)
                for (int r = 0; r < m; ++r) tmp[r * m + r] = tmp[r * m + r] + gamma;
            if (keep_block(tmp, (int64_t)m * n, eps, norm_kind))
                status = rowbuf_push(&rows[i], j, tmp, (int64_t)m * n);
            if (status != ORC_OK) break;
        }
    }
    if (status == ORC_OK)
        status = assemble(out, a->nbrows, a->nbcols, a->rbs, a->cbs, rows);
    free_rows(rows, a->nbrows);
    free(offa); free(offb); free(tmp);
    return status;
}

/* ------------------------------------------------------- sign iteration */

typedef struct {
    int32_t iterations;     /* number of X updates performed */
    int32_t n_multiplies;
    double r_hist[128];     /* r_k = ||X_k^2 - I||_F / n for k = 0..iterations */
    double scale;           /* s = ||H - mu I||_inf */
    double trace_x;
    double trace_p;         /* (n - trace X) / 2 */
    double flops;           /* sum over products of 2 m n k */
    int64_t nnzb_x[128];    /* stored blocks of X_k, k = 0..iterations (orc_sign only) */
    int64_t nnzb_y[128];    /* stored blocks of Y_k = filter(X_k X_k) (orc_sign only) */
} orc_sign_stats;

static double product_flops(const omat *a, const omat *b)
{
    double f = 0.0;
    for (int32_t i = 0; i < a->nbrows; ++i)
        for (int64_t ta = a->row_ptr[i]; ta < a->row_ptr[i + 1]; ++ta) {
            int32_t k = a->col_idx[ta];
            for (int64_t tb = b->row_ptr[k]; tb < b->row_ptr[k + 1]; ++tb)
                f += 2.0 * a->rbs[i] * a->cbs[k] * b->cbs[b->col_idx[tb]];
        }
    return f;
}

/*
 * Update X_{k+1} = X_k q(Y) / d from Y = X_k^2 for the iteration orders of
 * the Sign-Method section (Newton-Schulz, and the Pade-type iterations of
 * third and fifth order; Eq. fifth_order_sign), written with the OT/IR
 * refinement functions f_1, f_2 (Y = Z^2 for symmetric Z, S = I):
 *
 *   order 2:  X' = filter(1.5 X - 0.5 X Y)                      f_1 = Z(3 - Y)/2
 *   order 3:  W  = filter(3 Y Y + (15 I - 10 Y))
 *             X' = filter(X W / 8)                              f_2 = Z(15 - 10Y + 3Y^2)/8
 *   order 5:  Y2 = filter(Y Y)
 *             V  = filter(35 Y2 - 180 Y + 378 I)
 *             U  = filter(Y2 V + (315 I - 420 Y))
 *             X' = filter(X U / 128)                            Eq. fifth_order_sign
 *   order 7:  Y2 = filter(Y Y),  Y3 = filter(Y Y2)
 *             V  = filter(filter(231 Y3 - 1638 Y2 - 8580 I) + 5005 Y)
 *             C0 = filter(9009 Y2 - 6006 Y + 3003 I)
 *             U  = filter(Y3 V + C0)
 *             X' = filter(X U / 1024)
 *
 * The fifth-order form uses four multiplies per iteration (with the square
 * Y), as the Sign-Method section states; every product is filtered.  The
 * constant-plus-Y terms enter a multiply as its C_in.  The paper states that
 * the iterations go up to seventh order without printing that one; its
 * polynomial is the member of the printed family with g'(x) proportional to
 * (1 - x^2)^6 and g(1) = 1:
 * q(Y) = 3003 - 6006 Y + 9009 Y^2 - 8580 Y^3 + 5005 Y^4 - 1638 Y^5 + 231 Y^6,
 * evaluated as (3003 - 6006 Y + 9009 Y^2) + Y^3 (231 Y^3 - 1638 Y^2 + 5005 Y
 * - 8580) with five multiplies per iteration.
 */
static int sign_update(int32_t order, const omat *x, const omat *y, double eps, int norm_kind,
                       double tau, omat *xn, orc_sign_stats *st)
{
    omat c = {0}, w = {0}, y2 = {0}, v = {0};
    int status;
    if (order == 2) {
        st->flops += product_flops(x, y);
        st->n_multiplies++;
        return orc_multiply_screened(-0.5, x, y, 1.5, x, eps, norm_kind, tau, xn);
    }
    if (order == 3) {
        status = orc_shift_scale(y, 1.5, -10.0, &c);                  /* 15 I - 10 Y */
        if (status == ORC_OK) {
            st->flops += product_flops(y, y);
            st->n_multiplies++;
            status = orc_multiply(3.0, y, y, 1.0, &c, eps, norm_kind, &w);
        }
        if (status == ORC_OK) {
            st->flops += product_flops(x, &w);
            st->n_multiplies++;
            status = orc_multiply(0.125, x, &w, 0.0, NULL, eps, norm_kind, xn);
        }
        orc_free(&c); orc_free(&w);
        return status;
    }
    if (order == 7) {
        omat y3 = {0}, v1 = {0};
        st->flops += product_flops(y, y);
        st->n_multiplies++;
        status = orc_multiply(1.0, y, y, 0.0, NULL, eps, norm_kind, &y2);
        if (status == ORC_OK) {
            st->flops += product_flops(y, &y2);
            st->n_multiplies++;
            status = orc_multiply(1.0, y, &y2, 0.0, NULL, eps, norm_kind, &y3);
        }
        if (status == ORC_OK) status = orc_add(231.0, &y3, -1638.0, &y2, -8580.0, eps, norm_kind, &v1);
        if (status == ORC_OK) status = orc_add(1.0, &v1, 5005.0, y, 0.0, eps, norm_kind, &v);
        if (status == ORC_OK) status = orc_add(9009.0, &y2, -6006.0, y, 3003.0, eps, norm_kind, &c);
        if (status == ORC_OK) {
            st->flops += product_flops(&y3, &v);
            st->n_multiplies++;
            status = orc_multiply(1.0, &y3, &v, 1.0, &c, eps, norm_kind, &w);
        }
        if (status == ORC_OK) {
            st->flops += product_flops(x, &w);
            st->n_multiplies++;
            status = orc_multiply(1.0 / 1024.0, x, &w, 0.0, NULL, eps, norm_kind, xn);
        }
        orc_free(&c); orc_free(&w); orc_free(&y2); orc_free(&v); orc_free(&y3); orc_free(&v1);
        return status;
    }
    /* order 5 */
    st->flops += product_flops(y, y);
    st->n_multiplies++;
    status = orc_multiply(1.0, y, y, 0.0, NULL, eps, norm_kind, &y2);
    if (status == ORC_OK) status = orc_add(35.0, &y2, -180.0, y, 378.0, eps, norm_kind, &v);
    if (status == ORC_OK) status = orc_shift_scale(y, 0.75, -420.0, &c);   /* 315 I - 420 Y */
    if (status == ORC_OK) {
        st->flops += product_flops(&y2, &v);
        st->n_multiplies++;
        status = orc_multiply(1.0, &y2, &v, 1.0, &c, eps, norm_kind, &w);
    }
    if (status == ORC_OK) {
        st->flops += product_flops(x, &w);
        st->n_multiplies++;
        status = orc_multiply(1.0 / 128.0, x, &w, 0.0, NULL, eps, norm_kind, xn);
    }
    orc_free(&c); orc_free(&w); orc_free(&y2); orc_free(&v);
    return status;
}

/*
 * Matrix sign by the iterations of sign_update, and the density matrix
 * P = (I - sign(H - mu I)) / 2 with S = I (Sign-Method section, Eq. signdef
 * and the density-matrix relation):
 *
 *   s   = ||H - mu I||_inf               (scaling so the spectrum is in [-1, 1])
 *   X_0 = (H - mu I) / s                 (not filtered)
 *   for k = 0, 1, ...:
 *       Y   = filter(X_k X_k)
 *       r_k = ||Y - I||_F / n            (n = scalar dimension)
 *       stop if r_k < tol                 (or after fixed_iters updates)
 *       X_{k+1} = X_k q(Y) / d            (sign_update; order 2: 1.5 X - 0.5 X Y)
 *
 * Filtering after every product follows the Sign-Method section.  Returns the
 * last X (whose square was tested).  ORC_ENOCONV when r_k is not finite, when
 * r_k >= r_{k-1} three times in a row, or when max_iter updates did not reach
 * tol.
 */
int orc_sign(const omat *h, double mu, double eps, int norm_kind, double tol,
             int32_t max_iter, int32_t fixed_iters, int32_t order, double tau, omat *x_out,
             orc_sign_stats *st)
{
    if (h->nbrows != h->nbcols || eps < 0 || max_iter < 0 || max_iter > 120 ||
        fixed_iters < 0 || fixed_iters > 120 ||
        (order != 2 && order != 3 && order != 5 && order != 7) ||
        !(tau >= 0.0) || (tau > 0.0 && order != 2))
        return ORC_EINVAL;
    for (int32_t i = 0; i < h->nbrows; ++i) if (h->rbs[i] != h->cbs[i]) return ORC_EINVAL;
    memset(st, 0, sizeof(*st));
    double n = 0.0;
    for (int32_t i = 0; i < h->nbrows; ++i) n += h->rbs[i];

    double s = orc_inf_norm_shifted(h, mu);
    st->scale = s;
    if (!isfinite(s)) return ORC_ENONFINITE;
    if (s == 0.0) return ORC_ENOCONV;
    omat x = {0}, y = {0}, xn = {0};
    int status = orc_shift_scale(h, mu, 1.0 / s, &x);
    if (status != ORC_OK) return status;
    int stall = 0;
    for (int32_t k = 0;; ++k) {
        st->flops += product_flops(&x, &x);
        status = orc_multiply_screened(1.0, &x, &x, 0.0, NULL, eps, norm_kind, tau, &y);
        st->n_multiplies++;
        if (status != ORC_OK) break;
        st->nnzb_x[k] = x.nnzb;
        st->nnzb_y[k] = y.nnzb;
        double r = sqrt(orc_sqdist_identity(&y, 1.0)) / n;
        st->r_hist[k] = r;
        st->iterations = k;
        if (!isfinite(r)) { status = ORC_ENONFINITE; break; }
        if (fixed_iters > 0) {
            if (k == fixed_iters) break;
        } else {
            if (r < tol) break;
            if (k > 0 && r >= st->r_hist[k - 1]) { if (++stall >= 3) { status = ORC_ENOCONV; break; } }
            else stall = 0;
            if (k == max_iter) { status = ORC_ENOCONV; break; }
        }
        status = sign_update(order, &x, &y, eps, norm_kind, tau, &xn, st);
        orc_free(&y);
        if (status != ORC_OK) break;
        orc_free(&x);
        x = xn;
        memset(&xn, 0, sizeof(xn));
    }
    orc_free(&y);
    if (status == ORC_OK || status == ORC_ENOCONV) {
        st->trace_x = orc_trace(&x);
        st->trace_p = 0.5 * (n - st->trace_x);
    }
    *x_out = x;
    return status;
}

/* The second-order (Newton-Schulz) form of orc_sign. */
int orc_sign_ns(const omat *h, double mu, double eps, int norm_kind, double tol,
                int32_t max_iter, int32_t fixed_iters, omat *x_out, orc_sign_stats *st)
{
    return orc_sign(h, mu, eps, norm_kind, tol, max_iter, fixed_iters, 2, 0.0, x_out, st);
}

/* P = (I - X)/2 as a new matrix (inserts missing diagonal blocks). */
int orc_density_from_sign(const omat *x, omat *p)
{
    /* (I - X)/2 = -0.5 * (X - 1*I) */
    return orc_shift_scale(x, 1.0, -0.5, p);
}

/* ------------------------------------------- non-orthogonal basis (S != I) */

/*
 * S^{1/2} and S^{-1/2} of a symmetric positive definite S by the coupled
 * Newton-Schulz iteration: the second-order sign iteration applied to the
 * block matrix [[0, A], [I, 0]], whose sign is [[0, A^{1/2}], [A^{-1/2}, 0]]
 * (the relation of the Sign-Method section used for inverses and square
 * roots).  With X_k = [[0, Y_k], [Z_k, 0]] the update X(3I - X^2)/2 acts on
 * the two blocks; with T = Z Y:
 *
 *   s = ||S||_inf                         (Gershgorin bound: spectrum of S/s in (0, 1])
 *   Y_0 = S / s,  Z_0 = I
 *   for k = 0, 1, ...:
 *       T   = filter(Z_k Y_k)             (k = 0: T = Y_0, no product)
 *       r_k = ||T - I||_F / n;  stop if r_k < tol
 *       W   = 1.5 I - 0.5 T               (not filtered)
 *       Y_{k+1} = filter(Y_k W),  Z_{k+1} = filter(W Z_k)   (k = 0: Z_1 = W)
 *   S^{1/2} = sqrt(s) Y,  S^{-1/2} = Z / sqrt(s)
 *
 * The stall and max_iter rules are those of orc_sign; st->r_hist holds r_k,
 * st->scale holds s.  Both outputs are returned for OK and ENOCONV.
 */
int orc_sqrt_inv(const omat *s_in, double eps, int norm_kind, double tol, int32_t max_iter,
                 omat *sqrt_out, omat *isqrt_out, orc_sign_stats *st)
{
    if (s_in->nbrows != s_in->nbcols || eps < 0 || max_iter < 0 || max_iter > 120)
        return ORC_EINVAL;
    for (int32_t i = 0; i < s_in->nbrows; ++i) if (s_in->rbs[i] != s_in->cbs[i]) return ORC_EINVAL;
    memset(st, 0, sizeof(*st));
    double n = 0.0;
    for (int32_t i = 0; i < s_in->nbrows; ++i) n += s_in->rbs[i];
    const double sc = orc_inf_norm_shifted(s_in, 0.0);
    st->scale = sc;
    if (!isfinite(sc)) return ORC_ENONFINITE;
    if (sc == 0.0) return ORC_EINVAL;
    omat y = {0}, z = {0}, t = {0}, w = {0}, yn = {0}, zn = {0};
    int have_z = 0;                 /* Z_0 = I is implicit */
    int status = orc_shift_scale(s_in, 0.0, 1.0 / sc, &y);
    int stall = 0;
    for (int32_t k = 0; status == ORC_OK; ++k) {
        if (have_z) {
            st->flops += product_flops(&z, &y);
            st->n_multiplies++;
            status = orc_multiply(1.0, &z, &y, 0.0, NULL, eps, norm_kind, &t);
        } else {
            status = orc_shift_scale(&y, 0.0, 1.0, &t);     /* T_0 = Y_0 */
        }
        if (status != ORC_OK) break;
        const double r = sqrt(orc_sqdist_identity(&t, 1.0)) / n;
        st->r_hist[k] = r;
        st->iterations = k;
        if (!isfinite(r)) { status = ORC_ENONFINITE; break; }
        if (r < tol) break;
        if (k > 0 && r >= st->r_hist[k - 1]) { if (++stall >= 3) { status = ORC_ENOCONV; break; } }
        else stall = 0;
        if (k >= max_iter) { status = ORC_ENOCONV; break; }
        status = orc_shift_scale(&t, 3.0, -0.5, &w);          /* 1.5 I - 0.5 T */
        orc_free(&t);
        if (status == ORC_OK) {
            st->flops += product_flops(&y, &w);
            st->n_multiplies++;
            status = orc_multiply(1.0, &y, &w, 0.0, NULL, eps, norm_kind, &yn);
        }
        if (status == ORC_OK) {
            if (have_z) {
                st->flops += product_flops(&w, &z);
                st->n_multiplies++;
                status = orc_multiply(1.0, &w, &z, 0.0, NULL, eps, norm_kind, &zn);
            } else {
                zn = w;                                       /* Z_1 = W Z_0 = W */
                memset(&w, 0, sizeof(w));
            }
        }
        orc_free(&w);
        if (status != ORC_OK) break;
        orc_free(&y); orc_free(&z);
        y = yn; z = zn;
        memset(&yn, 0, sizeof(yn)); memset(&zn, 0, sizeof(zn));
        have_z = 1;
    }
    orc_free(&t); orc_free(&yn); orc_free(&zn);
    if (status == ORC_OK || status == ORC_ENOCONV) {
        int s2 = orc_shift_scale(&y, 0.0, sqrt(sc), sqrt_out);
        if (s2 == ORC_OK) {
            if (have_z) {
                s2 = orc_shift_scale(&z, 0.0, 1.0 / sqrt(sc), isqrt_out);
            } else {
                /* stopped at k = 0, Z_0 = I: I / sqrt(s) with only the diagonal
                   blocks, as (1/sqrt(s)) (E + I) of the empty matrix E */
                int64_t *rp = (int64_t *)calloc((size_t)s_in->nbrows + 1, sizeof(int64_t));
                if (!rp) {
                    s2 = ORC_ENOMEM;
                } else {
                    omat e = {s_in->nbrows, s_in->nbcols, s_in->rbs, s_in->cbs, 0, rp, NULL, NULL};
                    s2 = orc_shift_scale(&e, -1.0, 1.0 / sqrt(sc), isqrt_out);
                    free(rp);
                }
            }
        }
        if (s2 != ORC_OK) status = s2;
    }
    orc_free(&y); orc_free(&z);
    return status;
}

/*
 * Density matrix in a non-orthogonal basis, P = (I - sign(S^{-1} K - mu I))
 * S^{-1} / 2 (Sign-Method section, density relation), through its symmetric
 * form: with Z = S^{-1/2}, S^{-1} K - mu I = Z (K~ - mu I) Z^{-1} for
 * K~ = Z K Z, so sign(S^{-1} K - mu I) = Z sign(K~ - mu I) Z^{-1} and
 *
 *   P = Z (I - sign(K~ - mu I)) Z / 2.
 *
 * Steps: Z from orc_sqrt_inv (eps, tol, max_iter); K~ = filter(filter(Z K) Z);
 * X = orc_sign(K~, mu) of the given order; P~ = (I - X)/2;
 * P = filter(filter(Z P~) Z).  trace(P S) = trace(P~ Z S Z) = trace(P~) is
 * returned in *trace_ps.  Statuses: EINVAL for mismatched shapes; the first
 * non-OK status of the square root or the sign iteration (ENOCONV still
 * returns P).
 */
int orc_density_nonorth(const omat *k, const omat *s_in, double mu, double eps, int norm_kind,
                        double tol, int32_t max_iter, int32_t order, omat *p_out,
                        double *trace_ps, orc_sign_stats *st_sqrt, orc_sign_stats *st_sign)
{
    if (k->nbrows != s_in->nbrows || k->nbcols != s_in->nbcols) return ORC_EINVAL;
    for (int32_t i = 0; i < k->nbrows; ++i) if (k->rbs[i] != s_in->rbs[i]) return ORC_EINVAL;
    omat sq = {0}, z = {0}, k1 = {0}, kt = {0}, x = {0}, pt = {0}, p1 = {0};
    memset(st_sign, 0, sizeof(*st_sign));
    int status = orc_sqrt_inv(s_in, eps, norm_kind, tol, max_iter, &sq, &z, st_sqrt);
    int first = status;
    if (status == ORC_OK || status == ORC_ENOCONV)
        status = orc_multiply(1.0, &z, k, 0.0, NULL, eps, norm_kind, &k1);
    if (status == ORC_OK) status = orc_multiply(1.0, &k1, &z, 0.0, NULL, eps, norm_kind, &kt);
    if (status == ORC_OK) {
        status = orc_sign(&kt, mu, eps, norm_kind, tol, max_iter, 0, order, 0.0, &x, st_sign);
        if (first == ORC_OK) first = status;
    }
    if (status == ORC_OK || status == ORC_ENOCONV) {
        int s2 = orc_density_from_sign(&x, &pt);
        if (s2 == ORC_OK) { *trace_ps = orc_trace(&pt); s2 = orc_multiply(1.0, &z, &pt, 0.0, NULL, eps, norm_kind, &p1); }
        if (s2 == ORC_OK) s2 = orc_multiply(1.0, &p1, &z, 0.0, NULL, eps, norm_kind, p_out);
        status = (s2 == ORC_OK) ? first : s2;
    }
    orc_free(&sq); orc_free(&z); orc_free(&k1); orc_free(&kt); orc_free(&x); orc_free(&pt);
    orc_free(&p1);
    return status;
}

/* --------------------------------------------- canonical purification (TC2) */

typedef struct {
    int32_t iterations;     /* updates performed */
    int32_t n_multiplies;
    double e_hist[128];     /* e_k = (trace X_k - trace X_k^2) / n */
    int32_t branch[128];    /* update k: 0 = X^2, 1 = 2X - X^2, 2 = F + gamma G (TRS4) */
    double scale;           /* s = ||H||_inf */
    double trace_p;         /* trace of the returned P */
    double flops;
    double gamma_hist[128]; /* TRS4: gamma_k of update k (0 for TC2) */
} orc_tc2_stats;

/* Start shared by the purifications: checks, n, s = ||H||_inf and
 * X_0 = (s I - H) / (2 s), whose spectrum lies in [0, 1] with the low
 * energies near 1. */
static int purify_start(const omat *h, double eps, int32_t max_iter, orc_tc2_stats *st,
                        double *n_out, omat *x)
{
    if (h->nbrows != h->nbcols || eps < 0 || max_iter < 0 || max_iter > 120) return ORC_EINVAL;
    for (int32_t i = 0; i < h->nbrows; ++i) if (h->rbs[i] != h->cbs[i]) return ORC_EINVAL;
    memset(st, 0, sizeof(*st));
    double n = 0.0;
    for (int32_t i = 0; i < h->nbrows; ++i) n += h->rbs[i];
    *n_out = n;
    const double sc = orc_inf_norm_shifted(h, 0.0);
    st->scale = sc;
    if (!isfinite(sc)) return ORC_ENONFINITE;
    if (sc == 0.0) return ORC_EINVAL;
    return orc_shift_scale(h, sc, -0.5 / sc, x);
}

/* The TC2 map that raises the trace: filter(2 X - Y) with Y = X^2. */
static int tc2_raise(const omat *x, const omat *y, double eps, int norm_kind, omat *out)
{
    return orc_add(2.0, x, -1.0, y, 0.0, eps, norm_kind, out);
}

/*
 * Density matrix for a fixed occupation N by second-order trace-correcting
 * purification (TC2, one of the purifications the density-matrix paragraph
 * names), which needs no chemical potential (canonical ensemble):
 *
 *   s = ||H||_inf;  X_0 = (s I - H) / (2 s)        (spectrum in [0, 1], low energies near 1)
 *   for k = 0, 1, ...:
 *       Y   = filter(X_k X_k)
 *       e_k = (trace X_k - trace Y) / n;  stop if e_k < tol (returns X_k)
 *       X_{k+1} = Y                    if trace X_k > N   (lowers the trace)
 *               = filter(2 X_k - Y)    otherwise          (raises it)
 *
 * Both maps keep [0, 1] and push every eigenvalue to 0 or 1; the trace
 * test steers the count of those going to 1 towards N.  ORC_ENOCONV after
 * max_iter updates or when e_k is not finite (then ORC_ENONFINITE).
 */
int orc_tc2(const omat *h, double n_occ, double eps, int norm_kind, double tol, int32_t max_iter,
            omat *p_out, orc_tc2_stats *st)
{
    double n = 0.0;
    omat x = {0}, y = {0}, xn = {0};
    int status = purify_start(h, eps, max_iter, st, &n, &x);
    for (int32_t k = 0; status == ORC_OK; ++k) {
        st->flops += product_flops(&x, &x);
        st->n_multiplies++;
        status = orc_multiply(1.0, &x, &x, 0.0, NULL, eps, norm_kind, &y);
        if (status != ORC_OK) break;
        const double tx = orc_trace(&x), ty = orc_trace(&y);
        const double e = (tx - ty) / n;
        st->e_hist[k] = e;
        st->iterations = k;
        if (!isfinite(e)) { status = ORC_ENONFINITE; break; }
        if (e < tol) break;
        if (k >= max_iter) { status = ORC_ENOCONV; break; }
        if (tx > n_occ) {
            st->branch[k] = 0;
            orc_free(&x);
            x = y;
            memset(&y, 0, sizeof(y));
        } else {
            st->branch[k] = 1;
            status = tc2_raise(&x, &y, eps, norm_kind, &xn);
            orc_free(&y);
            if (status != ORC_OK) break;
            orc_free(&x);
            x = xn;
            memset(&xn, 0, sizeof(xn));
        }
    }
    orc_free(&y);
    if (status == ORC_OK || status == ORC_ENOCONV) st->trace_p = orc_trace(&x);
    *p_out = x;
    return status;
}

/*
 * Density matrix for a fixed occupation N by fourth-order trace-resetting
 * purification (TRS4, the other purification the density-matrix paragraph
 * names besides TC2 and the sign function).  Same start and stopping rule
 * as TC2; each update is the fourth-order map
 *
 *   F = X^2 (4X - 3X^2),  G = X^2 (I - X)^2,  X <- F + gamma G,
 *   gamma = (N - trace F) / trace G,
 *
 * which fixes 0 and 1 with zero slope for every gamma and, by the choice
 * of gamma, resets the trace to N.  It keeps [0, 1] only for gamma in
 * [0, 6]; outside, the TC2 maps move the trace instead:
 *
 *   for k = 0, 1, ...:
 *       Y = filter(X_k X_k);  e_k = (trace X_k - trace Y) / n;  stop if e_k < tol
 *       F = filter(Y filter(4 X_k - 3 Y))
 *       G = filter(D D) with D = filter(X_k - Y)       ((X - X^2)^2 = X^2 (I - X)^2)
 *       gamma = (N - trace F) / trace G, or 0 when the filter has removed all of G
 *       X_{k+1} = filter(2 X_k - Y) if gamma > 6;  Y if gamma < 0;  filter(F + gamma G) otherwise
 *
 * G vanishes only when X is idempotent to the filter's resolution; the
 * trace correction is then below that resolution too, and the update is F.
 * Three multiplies per update.  Status as orc_tc2.
 */
int orc_trs4(const omat *h, double n_occ, double eps, int norm_kind, double tol, int32_t max_iter,
             omat *p_out, orc_tc2_stats *st)
{
    double n = 0.0;
    omat x = {0}, y = {0}, w = {0}, f = {0}, d = {0}, g = {0}, xn = {0};
    int status = purify_start(h, eps, max_iter, st, &n, &x);
    for (int32_t k = 0; status == ORC_OK; ++k) {
        st->flops += product_flops(&x, &x);
        st->n_multiplies++;
        status = orc_multiply(1.0, &x, &x, 0.0, NULL, eps, norm_kind, &y);
        if (status != ORC_OK) break;
        const double tx = orc_trace(&x), ty = orc_trace(&y);
        const double e = (tx - ty) / n;
        st->e_hist[k] = e;
        st->iterations = k;
        if (!isfinite(e)) { status = ORC_ENONFINITE; break; }
        if (e < tol) break;
        if (k >= max_iter) { status = ORC_ENOCONV; break; }
        status = orc_add(4.0, &x, -3.0, &y, 0.0, eps, norm_kind, &w);
        if (status == ORC_OK) {
            st->flops += product_flops(&y, &w);
            st->n_multiplies++;
            status = orc_multiply(1.0, &y, &w, 0.0, NULL, eps, norm_kind, &f);
        }
        if (status == ORC_OK) status = orc_add(1.0, &x, -1.0, &y, 0.0, eps, norm_kind, &d);
        if (status == ORC_OK) {
            st->flops += product_flops(&d, &d);
            st->n_multiplies++;
            status = orc_multiply(1.0, &d, &d, 0.0, NULL, eps, norm_kind, &g);
        }
        orc_free(&w);
        orc_free(&d);
        if (status != ORC_OK) break;
        const double tf = orc_trace(&f), tg = orc_trace(&g);
        const double gamma = tg > 0.0 ? (n_occ - tf) / tg : 0.0;
        st->gamma_hist[k] = gamma;
        if (gamma > 6.0) {
            st->branch[k] = 1;
            status = tc2_raise(&x, &y, eps, norm_kind, &xn);
        } else if (gamma < 0.0) {
            st->branch[k] = 0;
            xn = y;
            memset(&y, 0, sizeof(y));
        } else {
            st->branch[k] = 2;
            status = orc_add(1.0, &f, gamma, &g, 0.0, eps, norm_kind, &xn);
        }
        orc_free(&y);
        orc_free(&f);
        orc_free(&g);
        if (status != ORC_OK) break;
        orc_free(&x);
        x = xn;
        memset(&xn, 0, sizeof(xn));
    }
    orc_free(&y);
    orc_free(&f);
    orc_free(&g);
    if (status == ORC_OK || status == ORC_ENOCONV) st->trace_p = orc_trace(&x);
    *p_out = x;
    return status;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the oracle's later parallel regions (timing only; the results
 * do not depend on it: every block row is summed by one thread). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
