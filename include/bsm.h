/*
 * bsm -- block-sparse matrix multiply and Newton-Schulz sign iteration on
 * AMD MI355X (gfx950).  C ABI: plain pointers and sizes, no C++ or torch
 * types.  Every call returns a bsm_status; on failure the handles passed in
 * are left unchanged and bsm_last_error() describes what went wrong.
 *
 * The operations follow the paper's statement of the problem:
 *   - blocked compressed-sparse-row (blocked CSR) matrices whose block sizes
 *     come from the atomic basis ("DBCSR library" section);
 *   - C = alpha*A*B + beta*C computed as products of small dense blocks
 *     ("Local multiplication" and "Batched execution" subsections);
 *   - after each product, blocks below eps_filter are flushed to zero to keep
 *     the matrix sparse ("Sign-Method" section);
 *   - sign(A) = A (A^2)^{-1/2} (Sign-Method, Eq. signdef) by Newton-Schulz
 *     iteration, and the density matrix P = (I - sign(H - mu I))/2 (the
 *     density-matrix relation of the same section, with S = I).
 *
 * Matrix layout (host or device arrays, as the on_device flag says):
 *   row_blk_size[nbrows], col_blk_size[nbcols]  int32, each in [1, 32],
 *                                                always host arrays;
 *   row_ptr[nbrows+1]  int64, row_ptr[0] = 0, non-decreasing, row_ptr[nbrows] = nnzb;
 *   col_idx[nnzb]      int32, in [0, nbcols), strictly increasing in each row;
 *   values             float64, the stored blocks concatenated in CSR order,
 *                      block (i,j) row-major with row_blk_size[i] rows and
 *                      col_blk_size[j] columns.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Work is queued on it; calls that must learn a size computed on
 * the device (the multiply, the filter, create from device arrays) wait for
 * the stream before they return, and so do calls that return host values.
 * Handles may be used from one thread at a time; a handle's memory lives on
 * the device that was current when it was created.
 *
 * Filter rule (the paper flushes "elements smaller than eps_filter"; read
 * here block by block): BSM_NORM_FROB drops block b iff sum(b_ij^2) <
 * eps^2, BSM_NORM_MAXABS drops it iff max|b_ij| < eps.  eps = 0 drops
 * nothing (exact-zero blocks are kept).
 */
#ifndef BSM_H
#define BSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsm_matrix_s *bsm_matrix;
typedef struct bsm_plan_s *bsm_plan;

typedef enum {
    BSM_OK = 0,
    BSM_EINVAL = -1,      /* bad argument, non-canonical matrix, size mismatch */
    BSM_ENOMEM = -2,      /* device allocation failed */
    BSM_EDEVICE = -3,     /* a HIP runtime call failed */
    BSM_ENOCONV = -4,     /* sign iteration did not reach tol */
    BSM_ENONFINITE = -5,  /* NaN or Inf met in a norm */
    BSM_ECAPACITY = -6    /* a fixed-capacity buffer was too small */
} bsm_status;

typedef enum {
    BSM_FP64 = 0,        /* block products in FP64 */
    BSM_FP32 = 1,        /* operands rounded to FP32, FP32 MFMA, FP32 accumulation per C block */
    BSM_SPLIT_BF16 = 2,  /* x = hi + lo in BF16, hi*hi + hi*lo + lo*hi on MFMA, FP32 accumulation
                            (about 17 significant bits per operand) */
    BSM_SPLIT_BF16X3 = 3 /* x = hi + mid + lo in BF16; the six products of the three parts whose
                            size is at least 2^-18 of hi*hi (hi*hi, hi*mid, mid*hi, hi*lo, lo*hi,
                            mid*mid) on MFMA, FP32 accumulation (about 26 bits per operand) */
} bsm_precision;

typedef enum { BSM_NORM_FROB = 0, BSM_NORM_MAXABS = 1 } bsm_norm;

typedef struct {
    int32_t nbrows, nbcols;
    int64_t nnzb;        /* stored blocks */
    int64_t nvalues;     /* stored scalars */
    int64_t nrows, ncols;/* scalar dimensions */
} bsm_info;

typedef struct {
    int64_t n_products;          /* block products A_ik*B_kj of the operands' patterns */
    double flops;                /* sum over products done of 2*m*n*k (screened ones left out) */
    int64_t nnzb_unfiltered;     /* stored blocks of the product before the filter */
    int64_t nnzb;                /* stored blocks of C after the filter */
    double smm_ms;               /* device time of the block-product kernels (HIP events) */
    double total_ms;             /* device time of the whole multiply (HIP events) */
    int32_t smm_launches;        /* number of block-product kernel launches */
    int32_t pad_;
    int64_t n_screened;          /* products left out by norm screening (of n_products) */
    double class_ms[16];         /* mixed sizes, one launch per (m, n) class: device time of
                                    class 4 c(m) + c(n), c = 0..3 for sizes 5, 13, 23, 26 */
} bsm_mult_stats;

typedef struct {
    double eps_filter;       /* filter threshold after every product (>= 0) */
    double tol;              /* stop when ||X^2 - I||_F / n < tol */
    int32_t max_iter;        /* at most this many X updates (<= 120) */
    int32_t fixed_iters;     /* > 0: exactly this many updates, tol ignored */
    int32_t norm;            /* bsm_norm of the filter */
    int32_t prec;            /* bsm_precision of the block products */
    int32_t fp64_final_iters;/* mixed precision: last updates done in FP64 */
    int32_t use_graph;       /* 1, 2: iterations from captured graphs (see bsm_sign_iterate) */
    double prec_switch_tol;  /* mixed precision: FP64 once r_k < this */
    int32_t order;           /* 2 (Newton-Schulz), 3, 5 or 7: see bsm_sign_iterate */
    int32_t pad_;
    double eps_screen;       /* > 0: product-level norm screening threshold (see
                                bsm_multiply_screened); order 2, FP64, no graph replay */
} bsm_sign_opts;

typedef struct {
    int32_t iterations;      /* X updates performed */
    int32_t n_multiplies;
    double r_hist[128];      /* r_k = ||X_k^2 - I||_F / n, k = 0..iterations */
    int32_t prec_hist[128];  /* precision of the products of update k */
    double scale;            /* s = ||H - mu I||_inf used for X_0 = (H - mu I)/s */
    double trace_x;          /* trace(X) of the returned iterate */
    double trace_p;          /* trace(P) = (n - trace X)/2 */
    double flops;            /* algorithmic flops of all block products */
    int64_t n_products;
    double smm_ms;           /* device time inside block-product kernels */
    double device_ms;        /* device time from first to last kernel (HIP events) */
    int64_t nnzb_final;      /* stored blocks of the returned X */
    int32_t graph_replays;   /* iterations run by replaying captured graphs */
    int32_t graph_fallbacks; /* replayed multiplies redone on the normal path: use_graph 1,
                                a capacity was exceeded; 2, the filter kept other blocks
                                (either: NaN/Inf appeared) */
    int32_t smm_launches;    /* block-product kernel launches of the counted multiplies */
    int32_t pad_;
    int64_t n_screened;      /* products left out by norm screening */
    int64_t nnzb_x_hist[128];/* stored blocks of X_k, k = 0..iterations */
    int64_t nnzb_y_hist[128];/* stored blocks of Y_k = filter(X_k X_k), k = 0..iterations */
    double class_ms[16];     /* bsm_mult_stats.class_ms summed over the multiplies */
} bsm_sign_stats;

/* Bisection record of bsm_mu_bisect. */
typedef struct bsm_mu_stats {
    int32_t steps;           /* sign iterations run (one per bisection midpoint) */
    int32_t sign_noconv;     /* midpoints whose sign iteration ended with BSM_ENOCONV */
    double mu_hist[64];      /* midpoint mu of step t */
    double count_hist[64];   /* trace(P) = (n - trace X)/2 at mu_hist[t] */
    double flops;            /* algorithmic flops of all block products */
    double device_ms;        /* summed device time of the sign iterations */
} bsm_mu_stats;

/* Record of bsm_tc2 and bsm_trs4. */
typedef struct bsm_tc2_stats {
    int32_t iterations;      /* updates performed */
    int32_t n_multiplies;
    double e_hist[128];      /* e_k = (trace X_k - trace X_k^2) / n, k = 0..iterations */
    int32_t branch[128];     /* update k: 0 = X^2, 1 = 2X - X^2, 2 = F + gamma G (TRS4) */
    double scale;            /* s = ||H||_inf */
    double trace_p;          /* trace of the returned P */
    double flops;            /* algorithmic flops of the block products */
    int64_t n_products;
    double smm_ms;           /* block-product kernel time (HIP events) */
    double device_ms;        /* device time of the whole call */
    double gamma_hist[128];  /* TRS4: gamma of update k (0 for TC2) */
} bsm_tc2_stats;

/* Record of bsm_submatrix_density. */
typedef struct bsm_sub_stats {
    int32_t n_sub;           /* submatrices (one per block column) */
    int32_t max_dim;         /* largest submatrix edge (scalars) */
    double mean_dim;         /* mean submatrix edge */
    int32_t max_iterations;  /* Newton-Schulz iterations of the slowest submatrix */
    int32_t n_batches;       /* batches the submatrices were processed in */
    double flops;            /* algorithmic flops of the dense products, 2 n^3 each */
    double gemm_ms;          /* device time of the dense product kernels (HIP events) */
    double device_ms;        /* device time of the whole call */
    double r_max;            /* largest final residual ||X^2 - I||_F / n over submatrices */
    int64_t nnzb;            /* stored blocks of P after the filter */
} bsm_sub_stats;

/* Default options: eps 0, tol 1e-6, max_iter 100, FROB, FP64, no graph, order 2,
 * no screening. */
void bsm_sign_opts_default(bsm_sign_opts *opts);

/*
 * Create a matrix by copying the arrays described above (the library never
 * aliases caller memory).  on_device = 1: row_ptr/col_idx/values are device
 * pointers on the current device; 0: host pointers.  The matrix is checked
 * for canonical form on the device; failures give BSM_EINVAL.  nnzb may be 0
 * (then row_ptr is all zeros and col_idx/values may be NULL).
 */
int bsm_create(bsm_matrix *out, int32_t nbrows, int32_t nbcols,
               const int32_t *row_blk_size, const int32_t *col_blk_size,
               int64_t nnzb, const int64_t *row_ptr, const int32_t *col_idx,
               const double *values, int on_device, void *stream);

/* Free the handle and its device memory (queued on the handle's last stream). */
int bsm_destroy(bsm_matrix m);

/* Sizes of the matrix (host values). */
int bsm_get_info(bsm_matrix m, bsm_info *info);

/*
 * Copy the matrix out into caller arrays of the sizes bsm_get_info gives
 * (row_ptr[nbrows+1], col_idx[nnzb], values[nvalues]); any pointer may be
 * NULL to skip that array.  on_device as in bsm_create.  Waits for the stream.
 */
int bsm_export(bsm_matrix m, int64_t *row_ptr, int32_t *col_idx, double *values,
               int on_device, void *stream);

/*
 * C = alpha * A * B + beta * C, then the filter (DBCSR multiply; Sign-Method
 * filtering).  The stored pattern of the result is every (i,j) with some k
 * having A_ik and B_kj stored, together with C's old pattern when beta != 0;
 * with beta == 0 C's old contents are ignored.  Blocks failing the filter
 * are then removed.  C is replaced (new pattern and values); it may be the
 * same handle as A or B.  A's column block sizes must equal B's row block
 * sizes, and C's block sizes must be A's rows by B's columns (BSM_EINVAL).
 * prec selects the arithmetic of the block products (bsm_precision); the
 * result, norms and filter are always FP64.  stats may be NULL.
 * BSM_ENONFINITE if a result block holds NaN or Inf (C is still replaced).
 */
int bsm_multiply(double alpha, bsm_matrix A, bsm_matrix B, double beta, bsm_matrix C,
                 double eps_filter, int32_t norm, int32_t prec,
                 bsm_mult_stats *stats, void *stream);

/*
 * C = alpha*A*B (beta = 0), then the filter, exactly as bsm_multiply, and a
 * plan of it: the multiply's symbolic results -- C's pattern, the product
 * lists or groups, their work order, the filter's keep-set -- kept in device
 * memory for numeric-only repeats with bsm_plan_execute (the DBCSR section's
 * Local multiplication: what is multiplied is decided apart from doing it).
 * *plan_out holds device memory until bsm_plan_destroy and refers to no
 * handle.  C may not be A or B (BSM_EINVAL); otherwise as bsm_multiply.
 */
int bsm_multiply_plan(double alpha, bsm_matrix A, bsm_matrix B, bsm_matrix C,
                      double eps_filter, int32_t norm, int32_t prec, bsm_plan *plan_out,
                      bsm_mult_stats *stats, void *stream);

/*
 * Numeric-only repeat of a planned multiply: C's values become alpha*A*B for
 * the current values of A and B (same kernels, so the same bits as
 * bsm_multiply), in the layout C got from bsm_multiply_plan.  Kernels only --
 * no allocation, copy or wait -- so the call may be captured into a hipGraph.
 * A and B must have the block patterns of the planning call and C its
 * result's pattern: block and scalar counts are checked (BSM_EINVAL), equal
 * positions are the caller's promise.  C may not be A or B.  Whether the
 * filter would now keep another block set, and whether a NaN/Inf appeared,
 * is recorded on the device for bsm_plan_status.  Executes of one plan share
 * its device state (work counters, unfiltered values, the record): on
 * different streams they must not overlap.
 */
int bsm_plan_execute(bsm_plan plan, bsm_matrix A, bsm_matrix B, bsm_matrix C, void *stream);

/*
 * Waits for stream and reports the executes since the last report:
 * *flags bit 0 = a result block held NaN or Inf, bit 1 = the filter would
 * have kept another block set (that result is the unfiltered product's kept
 * part, not a filtered product); then clears the record.
 */
int bsm_plan_status(bsm_plan plan, int32_t *flags, void *stream);

/*
 * Release a plan's device memory (NULL: no-op), in the order of the stream
 * of the plan's last call (as a matrix's arrays are released in the order
 * of its last stream): work queued on other streams that uses the plan must
 * be complete or ordered before that stream.
 */
int bsm_plan_destroy(bsm_plan plan);

/*
 * bsm_multiply with product-level norm screening (the Sign-Method section's
 * lever on the sparsity of the products): the term A_ik B_kj is left out of
 * C_ij when ||A_ik||_F^2 ||B_kj||_F^2 < eps_screen^2 (squared block norms in
 * FP64).  The stored pattern is that of the unscreened product (a block
 * whose terms were all left out holds beta C_in, or zeros, before the
 * filter); each C block's error is at most the sum of the left-out terms'
 * norm products, below (left-out terms) * eps_screen.  eps_screen = 0 is
 * bsm_multiply exactly.  FP64 only, uniform block sizes 5, 13, 23, 26 or 32
 * (the group kernel); else BSM_EINVAL.  stats->n_screened counts the
 * left-out products.
 */
int bsm_multiply_screened(double alpha, bsm_matrix A, bsm_matrix B, double beta, bsm_matrix C,
                          double eps_filter, int32_t norm, double eps_screen,
                          bsm_mult_stats *stats, void *stream);

/* Apply the filter to a matrix in place (same rule as after a multiply). */
int bsm_filter(bsm_matrix m, double eps_filter, int32_t norm, void *stream);

/*
 * Squared Frobenius norm of every stored block, in storage order, into the
 * device array out_dev[nnzb] (FP64; one wavefront reduction per block).
 */
int bsm_block_norms(bsm_matrix m, double *out_dev, void *stream);

/* trace(A) of a square block matrix (FP64, fixed summation order). Waits. */
int bsm_trace(bsm_matrix m, double *out, void *stream);

/* ||A - shift*I||_F^2 (missing diagonal blocks count as -shift*I). Waits. */
int bsm_sqdist_identity(bsm_matrix m, double shift, double *out, void *stream);

/*
 * bsm_sqdist_identity for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops): the same kernels and the
 * same summation order, so the same bits, written to the device double
 * *out_dev on `stream` without a wait.  Its per-block-row partial sums live
 * in a fixed device array of the library (2^20 doubles, 8 MiB per device,
 * held until the process ends) instead of allocated memory; nothing is
 * allocated or freed.  Calls that overlap on one device share that array
 * and race: order them on one stream.  The matrix must live on the current
 * device.  BSM_ECAPACITY for more than 2^20 block rows, BSM_EINVAL for a
 * non-square block matrix or NULL arguments.
 */
int bsm_sqdist_identity_noalloc(bsm_matrix m, double shift, double *out_dev, void *stream);

/*
 * out = scale * (A - mu*I) as a new handle (missing diagonal blocks are
 * inserted).  Also gives P = (I - X)/2 with mu = 1, scale = -1/2.
 */
int bsm_shift_scale(bsm_matrix A, double mu, double scale, bsm_matrix *out, void *stream);

/* max over scalar rows of sum_j |(A - mu I)_ij| (FP64). Waits. */
int bsm_inf_norm(bsm_matrix A, double mu, double *out, void *stream);

/*
 * Matrix sign of H - mu*I by second-order Newton-Schulz iteration
 * (Sign-Method section; Eq. signdef; the refinement function f_1 of the
 * OT/IR paragraph, X <- X(3I - X^2)/2):
 *   s = ||H - mu I||_inf;  X_0 = (H - mu I)/s;
 *   loop k: Y = filter(X_k X_k); r_k = ||Y - I||_F / n; stop if r_k < tol;
 *           X_{k+1} = filter(1.5 X_k - 0.5 X_k Y).
 * The returned X (new handle in *x_out, caller destroys) is the iterate
 * whose square was tested.  stats may be NULL.  BSM_ENOCONV if r_k is not
 * finite, grows three times in a row, or max_iter is reached (X is still
 * returned); BSM_ENONFINITE for NaN/Inf in H.
 * opts->order selects the update X_{k+1} = X_k q(Y)/d from Y = X_k^2 (the
 * Newton-Schulz and Pade-type iterations of the Sign-Method section, in the
 * form of the OT/IR refinement functions; every product filtered):
 *   2: X' = 1.5 X - 0.5 X Y                                   (2 multiplies)
 *   3: W = 3 Y Y + (15 I - 10 Y);  X' = X W / 8               (3 multiplies)
 *   5: Y2 = Y Y;  V = 35 Y2 - 180 Y + 378 I (bsm_add);
 *      U = Y2 V + (315 I - 420 Y);  X' = X U / 128            (4 multiplies,
 *      Eq. fifth_order_sign)
 *   7: Y2 = Y Y;  Y3 = Y Y2;  V = (231 Y3 - 1638 Y2 - 8580 I) + 5005 Y;
 *      C0 = 9009 Y2 - 6006 Y + 3003 I;  U = Y3 V + C0;  X' = X U / 1024
 *      (5 multiplies; the seventh order the section names, whose polynomial
 *      has g'(x) proportional to (1 - x^2)^6 like the printed ones)
 * Other orders: BSM_EINVAL.
 * opts->use_graph (order 2, no screening; the results are those of
 * use_graph = 0, bit for bit):
 *   1: with FP64 products and uniform block sizes 5, 6, 13, 23, 26 or 32 (or
 *      sizes in {5, 13, 23, 26} with every (m, n) class in one persistent
 *      launch, BSM_SMM_VARIANT=7), once an FP64 update has grown X's block
 *      count by at most half, iterations
 *      run from captured hipGraphs of the whole multiply (symbolic phase,
 *      block products, filter, residual), with every size kept in device
 *      memory and buffers of fixed capacity (sizes of the last iteration on
 *      the normal path times BSM_GRAPH_HEADROOM, default 1.25); two waits per
 *      iteration (r_k, then the update's record).  A multiply that overflows
 *      a capacity (or meets NaN/Inf) is redone on the normal path, which
 *      re-sizes the buffers; stats->graph_fallbacks counts these.  Other
 *      sizes and precisions: as 2.
 *   2: once an update leaves X's block pattern unchanged, the following
 *      iterations replay captured hipGraphs of the numeric kernels (one wait
 *      per iteration; no symbolic phase, allocation or compaction scan).  A
 *      replayed iteration whose filter would keep other blocks is redone on
 *      the normal path.
 */
int bsm_sign_iterate(bsm_matrix H, double mu, const bsm_sign_opts *opts,
                     bsm_matrix *x_out, bsm_sign_stats *stats, void *stream);

/*
 * C = alpha*A + beta*B + gamma*I, then the norm filter, as a new handle (the
 * matrix sum among the DBCSR operations of the DBCSR section).  B may be NULL
 * (treated as empty); otherwise A and B must have the same block sizes.
 * Pattern: pattern(A) union pattern(B), plus every diagonal block when
 * gamma != 0 (then A must be square with square diagonal blocks).  Per
 * element v = alpha*a + beta*b (absent blocks read as zero), then v += gamma
 * on the diagonal.  BSM_EINVAL for mismatched sizes, eps < 0 or non-finite
 * coefficients.
 */
int bsm_add(double alpha, bsm_matrix A, double beta, bsm_matrix B, double gamma,
            double eps_filter, int32_t norm, bsm_matrix *out, void *stream);

/*
 * Chemical potential for a fixed electron count (the canonical ensemble
 * that the Density-matrix-based-methods paragraph says sign purification
 * needs extra iterations for): bisection on mu for trace(P(mu)) =
 * (n - trace sign(H - mu I))/2, which does not decrease with mu.
 *   step t: mu = (lo + hi)/2; X = sign(H - mu I) (bsm_sign_iterate with opts);
 *           count = (n - trace X)/2;
 *           stop if |count - n_target| <= count_tol;
 *           else lo = mu if count < n_target, hi = mu otherwise.
 * The caller brackets the answer: count(mu_lo) <= n_target <= count(mu_hi)
 * (the endpoints themselves are never evaluated); mu_lo < mu_hi finite,
 * count_tol > 0, 1 <= max_steps <= 64, else BSM_EINVAL.  A midpoint whose
 * sign iteration ends with BSM_ENOCONV (mu near an eigenvalue) still gives
 * its count, and is counted in stats->sign_noconv.  Returns BSM_OK with the
 * accepted mu in *mu_out and its X in *x_out (new handle, caller destroys),
 * or BSM_ENOCONV after max_steps midpoints with the last mu and X; any other
 * error of the sign iteration is returned as is, with no X.  stats may be
 * NULL.  Blocks until the last count is known.
 */
int bsm_mu_bisect(bsm_matrix H, double n_target, double mu_lo, double mu_hi, double count_tol,
                  int32_t max_steps, const bsm_sign_opts *opts, double *mu_out,
                  bsm_matrix *x_out, bsm_mu_stats *stats, void *stream);

/*
 * S^{1/2} and S^{-1/2} of a symmetric positive definite S (non-orthogonal
 * basis) by the coupled Newton-Schulz iteration, i.e. the second-order sign
 * iteration on [[0, S], [I, 0]], whose sign is [[0, S^{1/2}], [S^{-1/2}, 0]]
 * (the Sign-Method section's relation for inverses and square roots):
 *   s = ||S||_inf;  Y_0 = S/s;  Z_0 = I;
 *   loop k: T = filter(Z_k Y_k) (k = 0: T = Y_0); r_k = ||T - I||_F / n;
 *           stop if r_k < tol;  W = 1.5 I - 0.5 T;
 *           Y_{k+1} = filter(Y_k W);  Z_{k+1} = filter(W Z_k) (k = 0: Z_1 = W);
 *   S^{1/2} = sqrt(s) Y,  S^{-1/2} = Z / sqrt(s).
 * opts: eps_filter, norm, tol, max_iter (0..120) are used (FP64 products).
 * stats (may be NULL): iterations, r_hist, scale = s, multiplies, flops.
 * Both results are new handles (caller destroys) for BSM_OK and BSM_ENOCONV
 * (r_k grew three times in a row or max_iter reached); BSM_EINVAL for a
 * non-square S or bad options, BSM_ENONFINITE for NaN/Inf.  Waits.
 */
int bsm_sqrt_inv(bsm_matrix S, const bsm_sign_opts *opts, bsm_matrix *sqrt_out,
                 bsm_matrix *isqrt_out, bsm_sign_stats *stats, void *stream);

/*
 * Density matrix in a non-orthogonal basis, P = (I - sign(S^{-1} K - mu I))
 * S^{-1} / 2 (Sign-Method section), through the symmetric form with
 * Z = S^{-1/2} (bsm_sqrt_inv): sign(S^{-1} K - mu I) = Z sign(Z K Z - mu I) Z^{-1},
 * so P = Z (I - sign(K~ - mu I)) Z / 2 with K~ = filter(filter(Z K) Z), the
 * sign by bsm_sign_iterate (opts, any order), and P = filter(filter(Z P~) Z).
 * *trace_ps (may be NULL) gets trace(P S) = trace(P~), the electron count.
 * sqrt_stats / sign_stats (may be NULL): the two iterations; sign_stats also
 * counts the four transform multiplies.  P is a new handle for BSM_OK and
 * BSM_ENOCONV (either iteration stopped early); BSM_EINVAL when K and S
 * differ in block sizes.  Waits.
 */
int bsm_density_nonorth(bsm_matrix K, bsm_matrix S, double mu, const bsm_sign_opts *opts,
                        bsm_matrix *p_out, double *trace_ps, bsm_sign_stats *sqrt_stats,
                        bsm_sign_stats *sign_stats, void *stream);

/*
 * Density matrix for a fixed occupation n_occ without a chemical potential,
 * by second-order trace-correcting purification (TC2, named among the
 * purifications of the density-matrix-based-methods paragraph):
 *   s = ||H||_inf;  X_0 = (s I - H)/(2s);
 *   loop k: Y = filter(X_k X_k); e_k = (trace X_k - trace Y)/n;
 *           stop if e_k < tol (P = X_k);
 *           X_{k+1} = Y if trace X_k > n_occ, else filter(2 X_k - Y).
 * opts: eps_filter, norm, tol, max_iter (0..120); FP64 products.  P is a new
 * handle (caller destroys) for BSM_OK and BSM_ENOCONV (max_iter reached);
 * BSM_ENONFINITE for NaN/Inf, BSM_EINVAL for a non-square H or bad options.
 * stats may be NULL.  Waits (two traces per iteration).
 */
int bsm_tc2(bsm_matrix H, double n_occ, const bsm_sign_opts *opts, bsm_matrix *p_out,
            bsm_tc2_stats *stats, void *stream);

/*
 * Density matrix for a fixed occupation n_occ by fourth-order
 * trace-resetting purification (TRS4, named with TC2 and the sign function
 * in the density-matrix-based-methods paragraph).  Same start and stopping
 * rule as bsm_tc2; each update
 *   F = filter(Y filter(4 X_k - 3 Y)), G = filter(D D), D = filter(X_k - Y),
 *   gamma = (N - trace F) / trace G   (0 when the filter has removed all of G),
 *   X_{k+1} = filter(2 X_k - Y) if gamma > 6; Y if gamma < 0;
 *             filter(F + gamma G) otherwise,
 * with Y = filter(X_k X_k): three multiplies per update.  Arguments, status
 * and ownership as bsm_tc2; stats->gamma_hist records gamma per update.
 */
int bsm_trs4(bsm_matrix H, double n_occ, const bsm_sign_opts *opts, bsm_matrix *p_out,
             bsm_tc2_stats *stats, void *stream);

/*
 * Density matrix by the submatrix method (section "Submatrix Method"): for
 * every block column j, the dense principal submatrix T_j of H over the
 * block rows stored in column j (ascending, j included), its density
 * matrix P_j = (I - sign(T_j - mu I))/2, and P's block column j = P_j's
 * block column of j, on H's pattern; P is then filtered (eps_filter, norm).
 * sign(T_j - mu I) by the dense Newton-Schulz iteration from
 * X_0 = (T_j - mu I)/||T_j - mu I||_inf, each submatrix stopped when
 * ||X^2 - I||_F / n_j < tol; FP64 throughout.
 * H: square, square diagonal blocks, every diagonal block stored, block
 * columns spanning at most 32768 rows.  opts: eps_filter, norm, tol,
 * max_iter (0..120); order, prec, graph and screening are ignored.  Device
 * memory: three dense padded squares per submatrix of a batch (batches of
 * consecutive columns up to 48 GiB, BSM_SUB_BATCH_BYTES).  P is a new
 * handle (caller destroys) for BSM_OK and BSM_ENOCONV (some submatrix
 * above tol after max_iter); BSM_ENONFINITE for NaN/Inf, BSM_EINVAL for bad
 * arguments.  stats may be NULL.  Waits (a residual read per iteration).
 */
int bsm_submatrix_density(bsm_matrix H, double mu, const bsm_sign_opts *opts, bsm_matrix *p_out,
                          bsm_sub_stats *stats, void *stream);

/*
 * B = A^T as a new handle (caller destroys): transpose, one of the
 * operations of the DBCSR library section.  Block (i, j) of A (m x n,
 * row-major) becomes block (j, i) of B (its n x m transpose); B's block
 * rows have A's column sizes and its block columns A's row sizes; columns
 * ascending in every row.  Any shape, including empty.  BSM_EINVAL for a
 * NULL argument.
 */
int bsm_transpose(bsm_matrix A, bsm_matrix *out, void *stream);

/* P = (I - X)/2 from a sign matrix X, as a new handle; trace_p (may be NULL) gets trace(P). */
int bsm_density_from_sign(bsm_matrix X, bsm_matrix *p_out, double *trace_p, void *stream);

/*
 * Autotuning support (the paper autotunes its block-product kernels per
 * (m, n, k), "Batched execution" subsection).  Kernel parameters of the
 * run-time-shape FP64 block-product kernel:
 *   family   0: 16x16x4 FP64 matrix-core tiles; 1: 4x4x4 (four blocks per
 *            instruction); 2: the (m, n)-specialised kernel (m, n in
 *            {5, 13, 23, 26}, k <= 26); 3: the compile-time-shape kernel
 *            (m = n = k in {5, 6, 13, 23, 26, 32});
 *   wpg      C blocks (wavefronts) per workgroup: 1, 2 or 4;
 *   prefetch 1: load the next product's operands while multiplying.
 */
typedef struct {
    int32_t family;
    int32_t wpg;
    int32_t prefetch;
    int32_t reserved;
} bsm_smm_params;

/*
 * Time n_params parameter sets on a synthetic stack: n_cblocks C blocks of
 * m x n, each with prods_per_cblock products A(m x k) * B(k x n) whose
 * operand blocks are drawn from pools of 1024 blocks (k = 0: the products
 * cycle through k = 5, 13, 23, 26).  ms_out[i] (host) gets the median kernel
 * time of `reps` runs of params[i].  Sizes 1..32; waits for the stream.
 */
int bsm_smm_bench(int32_t m, int32_t n, int32_t k, int64_t n_cblocks,
                  int32_t prods_per_cblock, int32_t n_params, const bsm_smm_params *params,
                  int32_t reps, double *ms_out, void *stream);

/*
 * Install kernel parameters for (m, n, k) triples (mnk holds 3 ints per
 * entry; k = 0 means "any k", used for the per-class launches of mixed
 * block sizes).  Later entries replace earlier ones; n_entries < 0 clears
 * the table.  Multiplies whose shapes have no entry use built-in choices.
 */
int bsm_set_smm_table(int32_t n_entries, const int32_t *mnk, const bsm_smm_params *params);

/* Message of the last failed call on this thread ("" if none). */
const char *bsm_last_error(void);

/* Library version string. */
const char *bsm_version(void);

/* The block-product kernel this thread launched last, with its template
 * arguments ("" before the first); for reports of what ran. */
const char *bsm_last_smm_kernel(void);

#ifdef __cplusplus
}
#endif

#endif /* BSM_H */
