/*
 * Sanitizer driver for the CPU oracle (test infrastructure only).
 *
 * Built together with bsm_oracle.c (included below, one translation unit)
 * under -fsanitize=address,undefined by tests/test_oracle_sanitize.py, it
 * calls every oracle entry point on small seeded matrices -- mixed block
 * sizes, empty rows, rectangular shapes, filters on both sides of zero, all
 * sign orders, the purifications, the square-root iteration and the
 * non-orthogonal density -- and frees every result, so that an
 * out-of-bounds access, a use after free, a leak or undefined behaviour in
 * the oracle ends the run with a sanitizer report.  Exit status 0 means
 * every call returned the status it should.
 */
#include <stdio.h>

#include "bsm_oracle.c"

static uint64_t rng_state;

/* SplitMix64 (Steele, Lea and Flood, 2014) */
static uint64_t next_u64(void)
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static double uniform01(void) { return (double)(next_u64() >> 11) * 0x1.0p-53; }
static double symmetric_unit(void) { return 2.0 * uniform01() - 1.0; }

/* owned matrix: the omat plus the block-size arrays it points at */
typedef struct {
    omat m;
    int32_t *rbs, *cbs;
} owned;

static void owned_free(owned *o)
{
    orc_free(&o->m);
    free(o->rbs);
    free(o->cbs);
}

static int32_t *sizes_from(const int32_t *src, int32_t n)
{
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int32_t i = 0; i < n; ++i) s[i] = src[i];
    return s;
}

/* every block position present with probability p, entries in [-1, 1] */
static owned random_bsr(int32_t nbr, int32_t nbc, const int32_t *rbs, const int32_t *cbs, double p)
{
    owned o;
    memset(&o, 0, sizeof(o));
    o.rbs = sizes_from(rbs, nbr);
    o.cbs = sizes_from(cbs, nbc);
    o.m.nbrows = nbr; o.m.nbcols = nbc; o.m.rbs = o.rbs; o.m.cbs = o.cbs;
    o.m.row_ptr = (int64_t *)calloc((size_t)nbr + 1, sizeof(int64_t));
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nbr * nbc + 1));
    int64_t nnzb = 0, nval = 0;
    for (int32_t i = 0; i < nbr; ++i) {
        for (int32_t j = 0; j < nbc; ++j)
            if (uniform01() < p) { ci[nnzb++] = j; nval += (int64_t)rbs[i] * cbs[j]; }
        o.m.row_ptr[i + 1] = nnzb;
    }
    o.m.nnzb = nnzb;
    o.m.col_idx = ci;
    o.m.values = (double *)malloc(sizeof(double) * (size_t)(nval ? nval : 1));
    for (int64_t t = 0; t < nval; ++t) o.m.values[t] = symmetric_unit();
    return o;
}

/* symmetric matrix on a symmetric random pattern with every diagonal block;
 * shift > 0: the diagonal gets -shift on the first n_occ orbitals of every
 * block and +shift on the rest after scaling so that shift exceeds every
 * row's absolute sum (a gap around 0) */
static owned symmetric_bsr(int32_t nb, const int32_t *sz, double p, double shift, double *n_occ)
{
    owned o;
    memset(&o, 0, sizeof(o));
    o.rbs = sizes_from(sz, nb);
    o.cbs = sizes_from(sz, nb);
    unsigned char *pat = (unsigned char *)calloc((size_t)nb * nb, 1);
    for (int32_t i = 0; i < nb; ++i) {
        pat[(size_t)i * nb + i] = 1;
        for (int32_t j = i + 1; j < nb; ++j)
            if (uniform01() < p) pat[(size_t)i * nb + j] = pat[(size_t)j * nb + i] = 1;
    }
    o.m.nbrows = o.m.nbcols = nb; o.m.rbs = o.rbs; o.m.cbs = o.cbs;
    o.m.row_ptr = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
    int64_t nnzb = 0, nval = 0;
    for (int32_t i = 0; i < nb; ++i) {
        for (int32_t j = 0; j < nb; ++j)
            if (pat[(size_t)i * nb + j]) { ++nnzb; nval += (int64_t)sz[i] * sz[j]; }
        o.m.row_ptr[i + 1] = nnzb;
    }
    o.m.nnzb = nnzb;
    o.m.col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)nnzb);
    o.m.values = (double *)malloc(sizeof(double) * (size_t)nval);
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnzb + 1));
    int64_t t = 0, v = 0;
    for (int32_t i = 0; i < nb; ++i)
        for (int32_t j = 0; j < nb; ++j)
            if (pat[(size_t)i * nb + j]) { o.m.col_idx[t] = j; off[t++] = v; v += (int64_t)sz[i] * sz[j]; }
    /* fill the upper triangle and the diagonal, mirror the rest */
    for (int32_t i = 0; i < nb; ++i)
        for (int64_t a = o.m.row_ptr[i]; a < o.m.row_ptr[i + 1]; ++a) {
            const int32_t j = o.m.col_idx[a];
            if (j < i) continue;
            double *blk = o.m.values + off[a];
            for (int r = 0; r < sz[i]; ++r)
                for (int c = 0; c < sz[j]; ++c)
                    blk[r * sz[j] + c] = (i == j && c < r) ? blk[c * sz[j] + r] : symmetric_unit();
            if (i == j) continue;
            int64_t b = o.m.row_ptr[j];
            while (o.m.col_idx[b] != i) ++b;
            double *mir = o.m.values + off[b];
            for (int r = 0; r < sz[i]; ++r)
                for (int c = 0; c < sz[j]; ++c) mir[c * sz[i] + r] = blk[r * sz[j] + c];
        }
    double big = 0.0;
    int64_t base = 0;
    for (int32_t i = 0; i < nb; ++i) {
        for (int r = 0; r < sz[i]; ++r) {
            double s = 0.0;
            for (int64_t a = o.m.row_ptr[i]; a < o.m.row_ptr[i + 1]; ++a) {
                const int32_t j = o.m.col_idx[a];
                for (int c = 0; c < sz[j]; ++c) s += fabs(o.m.values[off[a] + r * sz[j] + c]);
            }
            if (s > big) big = s;
        }
        base += sz[i];
    }
    *n_occ = 0.0;
    if (shift > 0.0)
        for (int32_t i = 0; i < nb; ++i) {
            int64_t a = o.m.row_ptr[i];
            while (o.m.col_idx[a] != i) ++a;
            const int occ = sz[i] / 4 + 1;
            for (int r = 0; r < sz[i]; ++r)
                o.m.values[off[a] + r * sz[i] + r] += (r < occ ? -1.0 : 1.0) * shift * 1.05 * big;
            *n_occ += occ;
        }
    free(off);
    free(pat);
    return o;
}

static int failures = 0;
static void expect(int got, int want, const char *what)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, got, want);
        ++failures;
    }
}

int main(void)
{
    rng_state = 12345u;
    omat out = {0}, out2 = {0};

    /* multiply, screened multiply, filter, transpose, add: mixed sizes, rectangular */
    const int32_t r1[7] = {5, 13, 1, 23, 26, 7, 32};
    const int32_t k1[5] = {4, 13, 26, 5, 9};
    const int32_t c1[6] = {23, 5, 13, 2, 26, 11};
    owned a = random_bsr(7, 5, r1, k1, 0.5);
    owned b = random_bsr(5, 6, k1, c1, 0.5);
    owned c = random_bsr(7, 6, r1, c1, 0.3);
    for (int norm = 0; norm < 2; ++norm)
        for (int e = 0; e < 3; ++e) {
            const double eps = e == 0 ? 0.0 : e == 1 ? 0.5 : 3.0;
            expect(orc_multiply(-0.5, &a.m, &b.m, 1.5, &c.m, eps, norm, &out), ORC_OK, "multiply");
            orc_free(&out);
            expect(orc_multiply(1.0, &a.m, &b.m, 0.0, NULL, eps, norm, &out), ORC_OK, "multiply beta 0");
            orc_free(&out);
            expect(orc_multiply_screened(1.0, &a.m, &b.m, 2.0, &c.m, eps, norm, 1.5, &out), ORC_OK,
                   "screened multiply");
            orc_free(&out);
            expect(orc_filter(&c.m, eps, norm, &out), ORC_OK, "filter");
            orc_free(&out);
            expect(orc_add(2.0, &c.m, -1.0, &c.m, 0.0, eps, norm, &out), ORC_OK, "add");
            orc_free(&out);
        }
    expect(orc_multiply(1.0, &a.m, &a.m, 0.0, NULL, 0.0, 0, &out), ORC_EINVAL, "mismatched multiply");
    expect(orc_filter(&c.m, -1.0, 0, &out), ORC_EINVAL, "negative eps");
    double *sq = (double *)malloc(sizeof(double) * (size_t)(c.m.nnzb + 1));
    expect(orc_block_sqnorms(&c.m, sq), ORC_OK, "block norms");
    free(sq);
    expect(orc_transpose(&c.m, &out), ORC_OK, "transpose");
    expect(orc_transpose(&out, &out2), ORC_OK, "transpose twice");
    orc_free(&out);
    orc_free(&out2);

    /* an empty matrix and a matrix with empty rows */
    const int32_t e1[3] = {3, 4, 5};
    owned z = random_bsr(3, 3, e1, e1, 0.0);
    expect(orc_multiply(1.0, &z.m, &z.m, 0.0, NULL, 0.0, 0, &out), ORC_OK, "empty multiply");
    orc_free(&out);
    expect(orc_transpose(&z.m, &out), ORC_OK, "empty transpose");
    orc_free(&out);
    (void)orc_trace(&z.m);
    (void)orc_sqdist_identity(&z.m, 1.0);
    (void)orc_inf_norm_shifted(&z.m, 0.5);
    expect(orc_shift_scale(&z.m, 0.5, 2.0, &out), ORC_OK, "shift of an empty matrix");
    orc_free(&out);

    /* sign iterations of every order, density, purifications, mu search parts */
    const int32_t s1[9] = {5, 13, 5, 23, 13, 5, 26, 5, 13};
    double n_occ = 0.0;
    owned h = symmetric_bsr(9, s1, 0.4, 1.0, &n_occ);
    orc_sign_stats st;
    const int orders[4] = {2, 3, 5, 7};
    for (int q = 0; q < 4; ++q) {
        expect(orc_sign(&h.m, 0.0, 1e-7, 0, 1e-9, 100, 0, orders[q], 0.0, &out, &st), ORC_OK, "sign");
        expect(orc_density_from_sign(&out, &out2), ORC_OK, "density from sign");
        orc_free(&out);
        orc_free(&out2);
    }
    expect(orc_sign(&h.m, 0.0, 1e-7, 1, 1e-9, 100, 4, 2, 1e-9, &out, &st), ORC_OK, "screened fixed sign");
    orc_free(&out);
    expect(orc_sign(&h.m, 0.0, 0.0, 0, 1e-9, 2, 0, 2, 0.0, &out, &st), ORC_ENOCONV, "sign max_iter");
    orc_free(&out);
    orc_tc2_stats ts;
    expect(orc_tc2(&h.m, n_occ, 1e-7, 0, 1e-9, 100, &out, &ts), ORC_OK, "tc2");
    orc_free(&out);
    expect(orc_trs4(&h.m, n_occ, 1e-7, 0, 1e-9, 100, &out, &ts), ORC_OK, "trs4");
    orc_free(&out);

    /* square roots and the non-orthogonal density: S = I + 0.3 N / max row sum */
    double unused = 0.0;
    owned s = symmetric_bsr(9, s1, 0.4, 0.0, &unused);
    double big = 0.0;
    {
        int64_t *off = block_offsets(&s.m);
        for (int32_t i = 0; i < 9; ++i)
            for (int r = 0; r < s1[i]; ++r) {
                double sum = 0.0;
                for (int64_t t = s.m.row_ptr[i]; t < s.m.row_ptr[i + 1]; ++t) {
                    const int32_t j = s.m.col_idx[t];
                    for (int cc = 0; cc < s1[j]; ++cc) sum += fabs(s.m.values[off[t] + r * s1[j] + cc]);
                }
                if (sum > big) big = sum;
            }
        for (int64_t t = 0; t < off[s.m.nnzb]; ++t) s.m.values[t] *= 0.3 / big;
        for (int32_t i = 0; i < 9; ++i) {
            int64_t t = s.m.row_ptr[i];
            while (s.m.col_idx[t] != i) ++t;
            for (int r = 0; r < s1[i]; ++r) s.m.values[off[t] + r * s1[i] + r] += 1.0;
        }
        free(off);
    }
    expect(orc_sqrt_inv(&s.m, 1e-9, 0, 1e-10, 100, &out, &out2, &st), ORC_OK, "sqrt_inv");
    orc_free(&out);
    orc_free(&out2);
    double tps = 0.0;
    orc_sign_stats st2;
    expect(orc_density_nonorth(&h.m, &s.m, 0.0, 1e-9, 0, 1e-9, 100, 2, &out, &tps, &st, &st2), ORC_OK,
           "non-orthogonal density");
    orc_free(&out);

    owned_free(&a); owned_free(&b); owned_free(&c); owned_free(&z); owned_free(&h); owned_free(&s);
    if (failures) {
        fprintf(stderr, "%d unexpected statuses\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: every call returned its expected status\n");
    return 0;
}
