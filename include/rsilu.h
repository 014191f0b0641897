/*
 * rsilu: row-splitting ILU preconditioned least squares on one AMD MI355X.
 *
 * Solves min ||b - A x||_2 for a sparse A (m x n, m >= n), the problem (1.1)
 * of Scott and Tuma, "Row-Splitting ILU Preconditioners for Sparse
 * Least-Squares Problems". Setup (rsilu_factor) runs on the host: it prescales
 * the columns of A to unit 2-norm (Section 5.1) and computes the rectangular
 * ILUP(p, tau) factorization with threshold partial pivoting by rows
 * (Algorithms 4, 5 and 6), which selects the square block A1 and returns
 *   P A D ~ [L1; L2] U                                            (3.8)
 * with D the column scaling, L1 unit lower triangular (n x n), L2 (m-n) x n
 * and U upper triangular. The solve (rsilu_solve) runs entirely on the GPU:
 * the left-preconditioned CGLS of Algorithm 1. Its preconditioning step
 * h = M^{-1} A^T r is evaluated in one of two forms (rsilu_params_t.form):
 *   - Algorithm 3 on the residual components (the default): u = r2 - Y r1,
 *     S^ w = u, y = r1 + Y^T w, L1 v = y, U h = v, with Y = L2 L1^{-1}
 *     applied implicitly and S^ = I, the dense S~ = I + Y Y^T, or no
 *     correction at all;
 *   - Algorithm 2 with k = n on z = A^T r: M_a = (L1 U)^T (L1 U) stands for
 *     C1 = A1^T A1 and A2 for its factored image L2 U, so that
 *     h = U^{-1} L1^{-1} (I - Y^T S^{-1} Y) L1^{-T} U^{-T} z; with the dense
 *     S~ this is (A~^T A~)^{-1} z for A~ = [L1; L2] U, and without the
 *     correction it is (L1 U)^{-1} (L1 U)^{-T} z. Either way M^{-1} is
 *     symmetric positive definite, which Algorithm 1 assumes of it.
 *
 * Conventions for every call
 *   - Indices are 0-based. Host arrays are owned by the caller and only read
 *     during the call; the library keeps its own copies.
 *   - Device pointers are HIP device memory owned by the caller. Work is
 *     enqueued on the caller's stream (0 = the null stream).
 *   - Internal coordinates: "pivot order" means row k of the permuted,
 *     prescaled matrix A_hat = P A D is original row perm[k]; positions
 *     0..n-1 form A1, positions n..m-1 form A2.
 *   - No call throws; errors are returned as rsilu_status_t. A handle may be
 *     used by one thread / one stream at a time; separate handles are
 *     independent.
 */
#ifndef RSILU_H
#define RSILU_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSILU_OK = 0,            /* success / converged */
    RSILU_NOT_CONVERGED = 1, /* maxit reached; x holds the last iterate */
    RSILU_BREAKDOWN = 2,     /* (q,q) = 0, rho = 0 or a non-finite scalar in
                                Algorithm 1, or a dense S~ that is not
                                numerically positive definite at setup */
    RSILU_EINVAL = -1,       /* invalid argument (shape, index, NaN/Inf, ...) */
    RSILU_ENOMEM = -2,       /* host allocation failed or device buffer too small */
    RSILU_EHIP = -3,         /* a HIP runtime call failed */
    RSILU_ESTATE = -4,       /* call out of order (e.g. solve before upload) */
    RSILU_EINTERNAL = -5     /* a kernel hit its internal wait bound */
} rsilu_status_t;

/* S^ used in step 2 of Algorithm 3 / M_b in step 3 of Algorithm 2
 * (Section 3.2). */
enum {
    RSILU_S_AUTO = -1,    /* dense when m - n <= 4096, identity otherwise */
    RSILU_S_IDENTITY = 0, /* S^ = I: w = u */
    RSILU_S_DENSE = 1,    /* S~ = I + Y Y^T assembled and Cholesky-factored once */
    RSILU_S_NONE = 2,     /* no A2 correction: w = 0, so that Algorithm 3 gives
                             h = U^{-1} L1^{-1} r1 and Algorithm 2 gives
                             h = M_a^{-1} z */
    RSILU_S_CHEB = 4,     /* M_b^{-1} = a fixed Chebyshev polynomial in S~ (an approximation
                             S^ of S~, Section 3.2): poly_degree steps of the Chebyshev
                             iteration on S~ w = u from w = 0 over [1, b], b = 1.05 times a
                             50-step power-iteration estimate of lambda_max(S~) taken at
                             setup. Linear in u and symmetric positive definite: the default
                             degree is the smallest even K with (b - 1) eps_K <= poly_delta,
                             eps_K = 1 / T_K((b+1)/(b-1)), so the Algorithm 2 operator times
                             A~^T A~ has its eigenvalues in [1 - poly_delta, 1 + poly_delta]
                             (A~ = [L1; Y~ L1] U with the explicit Y~, [L1; L2] U otherwise),
                             and an even degree keeps it positive definite beyond b. A degree
                             that misses that bound (a fixed poly_degree too low for the
                             interval, or the cap of 512) starts the iteration from omega u,
                             omega = 1 / (1 + eps_K), which keeps M_b^{-1} and the operator
                             positive definite (stats.cheb_scale). LSQR may use it. S~ products
                             as for RSILU_S_CG. FP64 or FP32 (with the explicit Y~); hybrid or
                             level schedule */
    RSILU_S_CG = 3        /* cg_steps steps of conjugate gradients on S~ w = u from
                             w = 0 (Section 3.2; Table 3(a) uses two), S~ applied
                             implicitly as d + L2 L1^{-1} L1^{-T} L2^T d, or as
                             d + Y~ (Y~^T d) with the explicit Y~ (RSILU_Y_EXPLICIT);
                             with cg_precond = RSILU_CG_JACOBI the steps are preconditioned
                             by D = diag(S~) = 1 + the squared row norms of the explicit Y~
                             (z = D^{-1} res, alpha = (res, z) / (p, S~ p), p = z + beta p);
                             FP64 with the hybrid or level schedule only */
};

/* Preconditioner of the CG steps on S~ (RSILU_S_CG). */
enum {
    RSILU_CG_NONE = 0,   /* plain CG (Table 3(a)) */
    RSILU_CG_JACOBI = 1  /* diag(S~), from the explicit Y~ (needs RSILU_Y_EXPLICIT) */
};

/* How Y~ = L2 L1^{-1} is applied (Section 3.2; rsilu_params_t.ystore).
 *   IMPLICIT: Y~ r = L2 (L1^{-1} r) and Y~^T w = L1^{-T} (L2^T w), one triangular
 *             sweep and one product each, so a product with S~ = I + Y~ Y~^T costs
 *             two sweeps.
 *   EXPLICIT: Y~ is computed at setup and stored as a sparse matrix: row i of Y~
 *             solves y L1 = (row i of L2) by back substitution with L1^T on a sparse
 *             right-hand side, positions finalised in descending order; a finished
 *             entry that is zero or smaller than ytau in magnitude is dropped before it
 *             propagates. Products with Y~, Y~^T and S~ are then sparse products, with no
 *             triangular sweep. Used with S^ = I, CG or none (EINVAL with the dense S~),
 *             FP64 or FP32, hybrid or level schedule. */
enum {
    RSILU_Y_IMPLICIT = 0,
    RSILU_Y_EXPLICIT = 1
};

/* Form of the preconditioning step of Algorithm 1 (see the top of this file). */
enum {
    RSILU_FORM_ALG3 = 0, /* Algorithm 3 on (r1, r2) (default) */
    RSILU_FORM_ALG2 = 1  /* Algorithm 2, k = n, on z = A^T r */
};

/* Krylov method of rsilu_solve (rsilu_params_t.krylov).
 *   PCGLS: Algorithm 1.
 *   LSQR:  LSQR (Paige and Saunders) on A_hat N with N N^T = M^{-1}, written so
 *          that only M^{-1} is applied; the same iterates as Algorithm 1 with
 *          that M in exact arithmetic (Section 1 notes the equivalence of CGLS
 *          and LSQR), usually better behaved in floating point. It needs a
 *          symmetric positive definite M^{-1}: the Algorithm 2 form with S^
 *          none, dense or Chebyshev (AUTO resolves to dense when m - n <= 4096
 *          in FP64 with Y~ implicit, else to none), and the hybrid or level
 *          schedule. Its stop test uses
 *          the recurrence ||A^T r|| = |phibar c| ||D^{-1} s||. */
enum {
    RSILU_KRYLOV_PCGLS = 0,
    RSILU_KRYLOV_LSQR = 1
};

/* Precision of the preconditioner (rsilu_params_t.precision). With FP32 the
 * factors L1, L2, U are stored in FP32 on the device and every step of
 * Algorithm 3 or Algorithm 2 runs in FP32 (its input converted from and its
 * output back to FP64); the products with A, the Krylov vectors, the
 * recurrence scalars, the norms and the exit residual stay FP64. FP32 needs
 * the hybrid or level schedule and S^ = I, none, or Chebyshev with the explicit
 * Y~ (EINVAL otherwise; AUTO resolves to I or none). */
enum {
    RSILU_PREC_FP64 = 0,
    RSILU_PREC_FP32 = 1
};

/* Schedule of the sparse triangular solves with L1, L1^T and U. */
enum {
    RSILU_TRSV_SYNCFREE = 0, /* one launch per solve; rows wait on their inputs */
    RSILU_TRSV_LEVELS = 1,   /* one launch per level of the dependency DAG */
    RSILU_TRSV_HYBRID = 2    /* wide levels one launch each; runs of narrow levels
                                swept by a single workgroup through LDS (default) */
};

/* Level scheme of the single-workgroup sweeps of the hybrid schedule. Every
 * scheme solves each row as rhs minus the sum of its products, times the
 * reciprocal diagonal; they differ in how the threads share the work and in
 * the order of the row sums (chunk order, or a tree over lanes). */
enum {
    RSILU_SWEEP_AUTO = 0,      /* per factor, from its rows' lengths: SEGMENTED when
                                  nearly every level's rows have at most 64 chunks,
                                  else TWO_PHASE (default) */
    RSILU_SWEEP_TWO_PHASE = 1, /* one 4-entry chunk and one row per thread; chunk sums
                                  through LDS, two barriers per level */
    RSILU_SWEEP_SEGMENTED = 2, /* one chunk per thread, a row's chunks on consecutive
                                  lanes of one 16-lane group (of one wavefront for
                                  rows of 17 to 64 chunks) summed by a segmented scan,
                                  one barrier per level (levels with a row of more
                                  than 64 chunks are solved as wide levels) */
    RSILU_SWEEP_ROWS = 3       /* one row per thread, its chunks loaded two at a time,
                                  one barrier per level */
};

typedef struct {
    int32_t p;        /* ILUP: at most p entries kept per column of L~ and of U~
                         above the diagonal (Algorithm 4); default 10 */
    double tau;       /* ILUP drop tolerance: entries with |v| < tau dropped; 1e-2 */
    double mu;        /* threshold pivoting parameter, 0 < mu <= 1 (Algorithm 5); 0.1 */
    double small;     /* pivots with |v| < small are modified (Algorithm 6); 1e-10 */
    int32_t colscale; /* 1: prescale columns to unit 2-norm (Section 5.1); 1 */
    int32_t smode;    /* RSILU_S_*; default RSILU_S_AUTO */
    int32_t maxit;    /* Algorithm 1 iteration limit; 2000 (Section 5.1) */
    int32_t trsv;     /* RSILU_TRSV_*; default RSILU_TRSV_HYBRID */
    int32_t poll;     /* iterations enqueued between host polls of the stop flag; 8 */
    int32_t form;     /* RSILU_FORM_*; default RSILU_FORM_ALG3 */
    int32_t precision; /* RSILU_PREC_*; default RSILU_PREC_FP64 */
    int32_t cg_steps;  /* CG steps of RSILU_S_CG, 1..256; default 2 */
    int32_t krylov;    /* RSILU_KRYLOV_*; default RSILU_KRYLOV_PCGLS */
    int32_t graph;     /* 1: the `poll` iterations between two polls are captured once
                          into a HIP graph (per upload) and replayed, one launch instead
                          of some 30 kernel launches per iteration; 0: launched one by
                          one. Profiling runs always launch one by one. Default 1. */
    int32_t sweep;     /* RSILU_SWEEP_*; default RSILU_SWEEP_AUTO */
    int32_t ystore;    /* RSILU_Y_*; default RSILU_Y_IMPLICIT */
    double ytau;       /* drop tolerance of the explicit Y~ (RSILU_Y_EXPLICIT): an entry of
                          Y~ that is zero or below ytau in magnitude when its substitution
                          step finishes is dropped and not propagated; 0 keeps every
                          nonzero (Y~ exact up to rounding); default 1e-2 */
    int32_t poly_degree; /* RSILU_S_CHEB: steps of the Chebyshev iteration, 1..512, or 0 to
                            choose the smallest even degree that meets poly_delta; default 0 */
    double poly_delta;   /* RSILU_S_CHEB: bound on the spread of the preconditioned spectrum
                            around 1 that the automatic degree meets, 0 < poly_delta < 1;
                            default 0.9 */
    int32_t cg_precond;  /* RSILU_CG_*: preconditioner of the CG steps on S~; default
                            RSILU_CG_NONE */
    int32_t reserved3;   /* 0 */
} rsilu_params_t;

typedef struct {
    int64_t m, n, nnz_a;   /* after stripping explicit zeros */
    int64_t nnz_l1;        /* strictly lower entries of L1 (unit diagonal implicit) */
    int64_t nnz_l2;        /* entries of L2 */
    int64_t nnz_u;         /* strictly upper entries of U (diagonal not counted) */
    int64_t psize;         /* nnz_l1 + nnz_l2 + nnz_u + n, plus (m-n)(m-n+1)/2
                              for the packed dense S~ (Tables 2 and 3) */
    int64_t nmod;          /* pivots modified by Algorithm 6 */
    int32_t levels_l1;     /* levels of the DAG of the L1 forward solve */
    int32_t levels_l1t;    /* ... of the L1^T backward solve */
    int32_t levels_u;      /* ... of the U backward solve */
    int32_t levels_ut;     /* ... of the U^T forward solve */
    int32_t smode;         /* S^ actually used (RSILU_S_IDENTITY, _DENSE, _NONE, _CG or _CHEB) */
    int32_t sweep_schemes; /* hybrid schedule: byte f (f = 0 L1, 1 L1^T, 2 U, 3 U^T) has bit s
                              set when a single-workgroup sweep of that factor uses level
                              scheme s (0 two phases, 1 segmented, 2 one row per thread, 3
                              segmented with rows of up to 64 chunks) and bit 7 when a level
                              of it is a multi-CU launch */
    size_t device_bytes;   /* what rsilu_upload needs */
    int64_t nnz_y;         /* entries of the explicit Y~ (0 when applied implicitly) */
    double cheb_b;         /* RSILU_S_CHEB: upper end b of the Chebyshev interval [1, b] */
    int32_t cheb_degree;   /* RSILU_S_CHEB: steps of the Chebyshev iteration (0: S~ = I) */
    int32_t reserved2;
    double cheb_scale;     /* RSILU_S_CHEB: omega, the scale of the iteration's input (1 when
                              the degree meets the poly_delta bound) */
} rsilu_stats_t;

typedef struct rsilu_ctx *rsilu_handle_t;

/* Defaults of rsilu_params_t: p = 10, tau = 1e-2, mu = 0.1, small = 1e-10
 * (Section 5.2 settings, with tau = 1e-2), colscale = 1, smode = AUTO,
 * maxit = 2000 (Section 5.1), trsv = HYBRID, poll = 8, form = ALG3,
 * precision = FP64, cg_steps = 2, krylov = PCGLS, graph = 1, sweep = AUTO,
 * ystore = IMPLICIT, ytau = 1e-2, poly_degree = 0, poly_delta = 0.9, cg_precond = NONE. */
void rsilu_params_default(rsilu_params_t *params);

/* Setup on the host (Section 5.1 prescaling; Algorithms 4-6; the splitting
 * (3.8); Section 3.2 dense S~ when requested).
 * A is given in CSR: rowptr[m+1] (int64), colind[nnz] (int32, sorted and
 * unique within each row), val[nnz] (finite FP64). Explicit zeros are
 * stripped. params may be NULL (defaults). On success *out owns a new handle
 * (free it with rsilu_destroy).
 * Errors: EINVAL for m < n, n < 1, bad pointers or indices, unsorted or
 * duplicated columns, non-finite values, invalid parameters, more than
 * 2^31 - 1 entries in a factor; ENOMEM when host memory runs out;
 * BREAKDOWN when the dense S~ is not numerically positive definite.
 * Rank deficiency is not an error: Algorithm 6 modifies the pivots and
 * stats.nmod counts them. */
rsilu_status_t rsilu_factor(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *colind,
                            const double *val, const rsilu_params_t *params, rsilu_handle_t *out);

/* Exact size in bytes of the device buffer rsilu_upload needs: operators,
 * level schedules, Krylov state and workspace. 0 for a NULL handle. */
size_t rsilu_device_bytes(rsilu_handle_t h);

/* Copy the operators into dev_buf (caller-owned device memory of at least
 * rsilu_device_bytes(h) bytes, 256-byte aligned; it must outlive every later
 * call on h) on the given stream, and wait for the copy to finish.
 * Errors: EINVAL (NULL handle or buffer, misaligned buffer), ENOMEM (bytes too
 * small), EHIP (runtime error). May be called again with another buffer. */
rsilu_status_t rsilu_upload(rsilu_handle_t h, void *dev_buf, size_t bytes, hipStream_t stream);

/* Append `count` rows to A without refactoring (Section 3.4, adding rows). The
 * rows (host CSR: rowptr[count + 1] from 0, sorted unique column indices in
 * [0, n), finite values; explicit zeros are stripped; copied) become rows
 * m, ..., m + count - 1 of A and join A2 at the end of the row order. L1, U and
 * the level schedules are kept; each new row a gets the L2 row l that solves
 * U^T l^T = (a D)^T (D the setup's column scaling) by forward substitution,
 * with entries |l_j| < tau or zero dropped. The products' plans and, in dense
 * mode, S~ are rebuilt. The device layout grows: the handle has no device
 * buffer afterwards, so call rsilu_device_bytes and rsilu_upload again before
 * the next solve (solves return ESTATE until then); b then has m + count
 * values. Errors: EINVAL (NULL handle, bad rows, too many rows or entries, or
 * dense S~ beyond its size limit; the handle is unchanged), ENOMEM, BREAKDOWN
 * (the rebuilt dense S~ is not positive definite; destroy the handle). The
 * update is only as good as the kept factorization: a row that makes A rank
 * deficient is not detected. */
rsilu_status_t rsilu_add_rows(rsilu_handle_t h, int64_t count, const int64_t *rowptr, const int32_t *colind,
                              const double *val);

/* Remove `count` rows of A without refactoring (Section 3.4, removing rows).
 * rows: host array of distinct row indices in the current numbering (copied);
 * the remaining rows keep their order and are numbered 0 .. m - count - 1, so b
 * has m - count values afterwards. The factorization is kept: removed rows of A2
 * leave L2 and S~ is refactored; removed rows of A1 join R, and the
 * preconditioner becomes the Woodbury update M^{-1} + M^{-1} R^T W^{-1} R M^{-1},
 * W = I - R M^{-1} R^T, over every A1 row removed so far (M^{-1} the Algorithm 2
 * operator; each application then costs two of them, a product with R and R^T
 * and a dense solve with W's Cholesky factor). Needs form ALG2, FP64, the dense
 * S~ and a level or hybrid schedule (the mode in which M approximates A^T A, not
 * only its A1 part). The handle has no device buffer afterwards: upload again
 * before the next solve. The batched kernel does not take such a handle.
 * Errors: EINVAL (NULL handle or rows, another configuration, a bad or repeated
 * index, fewer than n rows left, more than 4096 removed A1 rows; the handle is
 * unchanged), ENOMEM, BREAKDOWN (S~ or W not positive definite: the removal
 * leaves the kept factorization without a usable preconditioner; destroy the
 * handle). */
rsilu_status_t rsilu_remove_rows(rsilu_handle_t h, int64_t count, const int64_t *rows);

/* Setup statistics (Tables 2 and 3 report psize and nmod). */
rsilu_status_t rsilu_get_stats(rsilu_handle_t h, rsilu_stats_t *stats);

/* perm[m]: original row index at each position of the ILUP row permutation
 * (Algorithm 4 interchanges). Host array owned by the caller. */
rsilu_status_t rsilu_get_perm(rsilu_handle_t h, int32_t *perm);

/* colnorm[n]: the 2-norms of the columns of A (1 for an empty column, or all
 * ones without prescaling); A_hat = P A diag(1/colnorm). */
rsilu_status_t rsilu_get_colnorm(rsilu_handle_t h, double *colnorm);

/* Factor and operator export, for inspection and tests (host arrays).
 * which: 0 = L1 (n x n, strictly lower), 1 = L2 ((m-n) x n),
 *        2 = U (n x n, strictly upper), 3 = A_hat (m x n, pivot order),
 *        4 = diagonal of U (val[n] only; rowptr and col may be NULL),
 *        5 = the explicit Y~ ((m-n) x n; RSILU_Y_EXPLICIT only, else EINVAL / -1).
 * rsilu_factor_nnz returns the entry count of `which` (or -1 if invalid).
 * rowptr has nrows+1 entries; columns are sorted within each row. */
int64_t rsilu_factor_nnz(rsilu_handle_t h, int32_t which);
rsilu_status_t rsilu_get_factor(rsilu_handle_t h, int32_t which, int64_t *rowptr, int32_t *col,
                                double *val);

/* Level schedule of a triangular solve: which = 0 L1 (forward), 1 L1^T
 * (backward), 2 U (backward), 3 U^T (forward). level_ptr[nlev+1] and
 * level_rows[n]; rows are ascending inside a level; nlev is in the stats. */
rsilu_status_t rsilu_get_levels(rsilu_handle_t h, int32_t which, int32_t *level_ptr,
                                int32_t *level_rows);

/* Algorithm 1 with the configured preconditioning form (after rsilu_upload).
 * b_dev[m]: the right-hand side in the original row order (device, read only).
 * x_dev[n]: the solution in the user's coordinates (device, written); must not
 * alias b_dev. Starts from x = 0 and stops when ||A^T r|| <= tol ||A^T b||
 * (on the user's A) or after maxit iterations.
 * Host outputs (each may be NULL): *iters, *atr_norm = ||A^T (b - A x)|| and
 * *atr_rel = atr_norm / ||A^T b||, both recomputed from x at exit.
 * Returns OK, NOT_CONVERGED, BREAKDOWN (x holds the last finite iterate's
 * update), EINVAL, ESTATE, EHIP or EINTERNAL. Blocks until the results are on
 * the host; all device work is on `stream`. If ||A^T b|| = 0 then x = 0,
 * iters = 0 and OK. */
rsilu_status_t rsilu_solve(rsilu_handle_t h, const double *b_dev, double tol, double *x_dev,
                           int32_t *iters, double *atr_norm, double *atr_rel, hipStream_t stream);

/* The steps of one iteration, on caller-owned device vectors in internal
 * coordinates, enqueued asynchronously on `stream` (after rsilu_upload).
 *
 * rsilu_spmv, op: 0  y[m] = A_hat x[n]        (Algorithm 1, q = A p)
 *                 1  y[n] = A_hat^T x[m]      (Algorithm 1, z = A^T r)
 *                 2  y[m-n] = L2 x[n]         (Algorithm 3, Y r1 = L2 L1^{-1} r1)
 *                 3  y[n] = L2^T x[m-n]       (Algorithm 3, Y^T w = L1^{-T} L2^T w)
 *                 4  y[m-n] = Y~ x[n]         (the explicit Y~, RSILU_Y_EXPLICIT only)
 *                 5  y[n] = Y~^T x[m-n]       (its transpose)
 * rsilu_trsv, which: 0  L1 x = rhs   1  L1^T x = rhs   2  U x = rhs
 *                   3  U^T x = rhs (Algorithm 2, M_a = (L1 U)^T (L1 U))  (n-vectors)
 * rsilu_apply:   h[n] from the residual r[m] by Algorithm 3.
 * rsilu_apply_z: h[n] = M^{-1} z[n] by Algorithm 2 (k = n, as above).
 * Both use the handle's S^ mode, whatever its form.
 * x and y (rhs and x) must not alias. EINVAL for a bad op/which or NULL. */
rsilu_status_t rsilu_spmv(rsilu_handle_t h, int32_t op, const double *x_dev, double *y_dev,
                          hipStream_t stream);
rsilu_status_t rsilu_trsv(rsilu_handle_t h, int32_t which, const double *rhs_dev, double *x_dev,
                          hipStream_t stream);
rsilu_status_t rsilu_apply(rsilu_handle_t h, const double *r_dev, double *h_dev, hipStream_t stream);
rsilu_status_t rsilu_apply_z(rsilu_handle_t h, const double *z_dev, double *h_dev, hipStream_t stream);

/* Kernel timing with HIP events recorded on the solve's stream, accumulated
 * over all rsilu_solve calls made while enabled (rsilu_set_profiling resets
 * the counters). Classes 0-8 time whole steps of an iteration (a triangular
 * solve is several kernel launches); classes 9-11 time single kernels, one
 * event pair per launch, and their `bytes` are the algorithmic bytes of the
 * timed launches: every stored value (8 B) and index (4 B) of the rows they
 * solve read once, and each row's right-hand side, result (and fused
 * addend and sum) once. */
enum {
    RSILU_PROF_SPMV_A = 0,    /* q = A_hat p (with its norm partials) */
    RSILU_PROF_SPMV_AT = 1,   /* z = A_hat^T r (with its norm partials) */
    RSILU_PROF_TRSV_L1 = 2,   /* L1 forward solves */
    RSILU_PROF_TRSV_L1T = 3,  /* L1^T backward solves */
    RSILU_PROF_TRSV_U = 4,    /* U backward solves */
    RSILU_PROF_SPMV_L2 = 5,   /* products with L2 (or with the explicit Y~) */
    RSILU_PROF_SPMV_L2T = 6,  /* products with L2^T (or with the explicit Y~^T) */
    RSILU_PROF_DENSE_S = 7,   /* dense S~ solves, or the CG steps on S~ (whole) */
    RSILU_PROF_TRSV_UT = 8,   /* U^T forward solves (Algorithm 2 form) */
    RSILU_PROF_K_SWEEP = 9,   /* launches of the single-workgroup sweep kernel */
    RSILU_PROF_K_LEVEL = 10,  /* launches of the one-level kernel (hybrid schedule) */
    RSILU_PROF_K_GATHER = 11, /* level-order gathers ahead of the sweeps */
    RSILU_PROF_K_SPMV_Y = 12, /* launches of the products with the explicit Y~ and Y~^T
                                 (inside and outside the CG steps on S~) */
    RSILU_PROF_COUNT = 13
};

typedef struct {
    int64_t launches[RSILU_PROF_COUNT];
    double ms[RSILU_PROF_COUNT];
    double bytes[RSILU_PROF_COUNT]; /* algorithmic bytes (kernel classes only) */
} rsilu_profile_t;

rsilu_status_t rsilu_set_profiling(rsilu_handle_t h, int32_t enable);
/* The same with only the classes whose bit is set in `mask` timed (bit i: class i; 0 turns
 * profiling off; rsilu_set_profiling(h, 1) sets every bit). Each timed launch group adds two
 * event records to the stream, so timing only the classes a caller needs keeps the solve's
 * own time close to that of an unprofiled solve. Resets the counters like
 * rsilu_set_profiling; EINVAL for a NULL handle or a bit at or above RSILU_PROF_COUNT. */
rsilu_status_t rsilu_set_profiling_mask(rsilu_handle_t h, uint32_t mask);
rsilu_status_t rsilu_get_profile(rsilu_handle_t h, rsilu_profile_t *out);

/* Release the handle's host memory and any HIP objects it created (not the
 * caller's device buffer). NULL is ignored. */
void rsilu_destroy(rsilu_handle_t h);

/* Static description of a status code. */
const char *rsilu_status_string(rsilu_status_t status);

#ifdef __cplusplus
}
#endif

#endif /* RSILU_H */
