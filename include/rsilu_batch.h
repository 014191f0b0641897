/*
 * rsilu batched persistent solves and their autotuner.
 *
 * rsilu_batch_solve advances many independent least-squares solves in ONE
 * kernel launch: each problem is owned by one workgroup, which runs the whole
 * preconditioned LSQR of that problem (initialisation, every iteration, the
 * exit residual) without leaving the kernel. Within the workgroup, the products
 * with A_hat and A_hat^T, the four triangular solves of the preconditioner
 * (level by level, one workgroup barrier per level) and the vector updates and
 * norms are separated by workgroup barriers only; no problem ever waits for
 * another, so every workgroup exits after at most maxit iterations.
 *
 * The arithmetic is that of rsilu_solve with krylov = RSILU_KRYLOV_LSQR and form =
 * RSILU_FORM_ALG2 (Algorithm 2 with k = n; LSQR in the M-inner-product form,
 * rsilu.h), with S^ none (no M_b correction, M^{-1} = (L1 U)^{-1} (L1 U)^{-T},
 * Section 3.1) or, with the explicit Y~ (ystore = RSILU_Y_EXPLICIT), the M_b
 * correction of Section 3.2 with M_b = I (RSILU_S_IDENTITY) or the Chebyshev
 * polynomial in S~ (RSILU_S_CHEB), whose steps the workgroup runs between the
 * L1^T and L1 solves; in the handle's preconditioner precision (FP64 or FP32; the
 * LSQR vectors, recurrences, norms and the exit residual stay FP64). Only the
 * order of the floating-point sums differs from rsilu_solve. A problem's result
 * depends only on its own data and on the tile, never on the other problems of
 * the launch.
 *
 * The batch object keeps the device descriptor table and captures, per
 * (count, tile), the descriptor upload, the launch and the result download into
 * a HIP graph that later calls replay.
 *
 * The autotuner (rsilu_tune) times every compiled tile, and the plain
 * multi-kernel path (rsilu_solve), on a few iterations of a given problem and
 * keeps its choice per problem signature (precision, size and density
 * classes, level-count class, long rows, the correction's cost class), so
 * later problems of the same class are not
 * timed again.
 *
 * All calls return rsilu_status_t; none throws.
 */
#ifndef RSILU_BATCH_H
#define RSILU_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "rsilu.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsilu_batch *rsilu_batch_t;
typedef struct rsilu_tuner *rsilu_tuner_t;

/* Tile of the persistent kernel: threads per workgroup (256, 512 or 1024),
 * lanes per row in the products with A_hat and A_hat^T (4 or 8) and in the
 * triangular solves (1 or 4). rsilu_batch_tiles lists the compiled ones. */
typedef struct {
    int32_t threads;
    int32_t spmv_lanes;
    int32_t tri_lanes;
    int32_t reserved; /* 0 */
} rsilu_tile_t;

/* Per-problem outcome of a batched solve (the outputs of rsilu_solve). */
typedef struct {
    int32_t status;   /* rsilu_status_t: OK, NOT_CONVERGED or BREAKDOWN */
    int32_t iters;
    double atr_norm;  /* true ||A^T (b - A x)||, recomputed at exit */
    double atr_rel;   /* atr_norm / ||A^T b|| */
} rsilu_batch_result_t;

/* Number of compiled tiles; when `tiles` is not NULL, the first `max` of them are
 * copied there. */
int32_t rsilu_batch_tiles(rsilu_tile_t *tiles, int32_t max);

/* 1 when the batched kernel takes h's configuration (LSQR, Algorithm 2 form, no
 * removed rows, and no M_b correction or the Chebyshev one through the explicit
 * Y~), 0 otherwise (also for NULL). h need not be uploaded. */
int32_t rsilu_batch_accepts(rsilu_handle_t h);

/* Create a batch object for up to `capacity` problems per launch on the current
 * device (allocates the descriptor table and pinned host mirrors).
 * EINVAL: capacity < 1 or > 65535; ENOMEM / EHIP on allocation failure. */
rsilu_status_t rsilu_batch_create(int32_t capacity, rsilu_batch_t *out);

/* Solve `count` problems in one launch on stream s and wait for it.
 *   hs[i]   uploaded handles, pairwise distinct, created with krylov = LSQR,
 *           form = ALG2 and S^ none (smode NONE, or AUTO resolved to none);
 *   b[i]    device pointer to the m_i right-hand-side values (user row order);
 *   tol[i]  stop when the LSQR estimate of ||A^T r|| <= tol[i] ||A^T b||;
 *   x[i]    device pointer receiving the n_i solution values (may not alias b[i]);
 *   tile    a compiled tile (rsilu_batch_tiles); NULL picks 1024 threads, 4 and 4 lanes;
 *   res[i]  host outcome of problem i.
 * Each handle's maxit bounds its iterations. A handle's work vectors are used, so
 * a handle may not be solved elsewhere while the call runs.
 * EINVAL: count outside [0, capacity], a NULL pointer, a handle not uploaded or
 * configured otherwise (another Krylov method or form, removed rows, or a
 * correction other than those above: dense S~, CG steps, or Y~ applied by
 * sweeps), a repeated handle, a tile that is not compiled, a
 * negative or non-finite tol; ESTATE: handles on another device than the
 * batch object; EHIP on runtime errors. count = 0 returns OK at once. */
rsilu_status_t rsilu_batch_solve(rsilu_batch_t bt, int32_t count, const rsilu_handle_t *hs,
                                 const double *const *b, const double *tol, double *const *x,
                                 const rsilu_tile_t *tile, rsilu_batch_result_t *res, hipStream_t s);

/* Free the batch object (NULL is ignored). Wait for its last launch first. */
void rsilu_batch_destroy(rsilu_batch_t bt);

/* For callers that cannot allocate device or pinned memory (code between stream
 * captures, tight serving loops, harnesses that forbid allocation): the batched
 * solve of rsilu_batch_solve without a batch object. The descriptor table and the
 * outcome slots of the launch live in a fixed device array of the library, one per
 * GPU (sizeof of 256 descriptors and outcomes, under 200 KiB), held until the process
 * ends; the call makes no hipMalloc, hipHostMalloc, hipFree or graph, and stages
 * the table through fixed host arrays of the library. Arguments, arithmetic, results
 * and errors as rsilu_batch_solve (each handle's maxit applies), with count at most
 * rsilu_batch_static_max() = 256 (EINVAL beyond) on the current device (ESTATE for
 * handles uploaded on another). It waits for its launch. Calls in one process are
 * serialised; calls from several processes on one GPU each use their own copy of the
 * array. */
rsilu_status_t rsilu_batch_solve_static(int32_t count, const rsilu_handle_t *hs, const double *const *b,
                                        const double *tol, double *const *x, const rsilu_tile_t *tile,
                                        rsilu_batch_result_t *res, hipStream_t s);
int32_t rsilu_batch_static_max(void);

/* Outcome of rsilu_tune. path: 0 = the persistent batched kernel with `tile`,
 * 1 = the plain multi-kernel path (rsilu_solve). The times are per iteration,
 * measured (or those of the cached measurement when from_cache = 1). */
typedef struct {
    int32_t path;
    int32_t from_cache;
    rsilu_tile_t tile;
    double batched_ms_per_iter;
    double plain_ms_per_iter;
} rsilu_tune_result_t;

/* Create an autotuner. A problem goes to the batched kernel when its best tile's
 * time per iteration is at most `slack` times that of the plain path (slack >= 1
 * favours the batched kernel, which leaves every other compute unit to the other
 * problems of its launch). `iters` (>= 2) iterations are timed per candidate:
 * the plain path (after one untimed run), the default tile, and the other tiles
 * only when the default one is within twice the slack of the plain path.
 * EINVAL: slack not finite or <= 0, iters < 2. */
rsilu_status_t rsilu_tuner_create(double slack, int32_t iters, rsilu_tuner_t *out);

/* Choose the path and tile for the uploaded handle h (configured as for
 * rsilu_batch_solve), timing candidates on stream s with the right-hand side
 * b_dev (m values) and writing scratch solutions into x_dev (n values). A problem
 * whose signature was tuned before reuses that choice (from_cache = 1) without
 * running anything. Calls on one tuner are serialised; h itself may not be in use
 * elsewhere during the call (its maxit is lowered while the plain path is
 * timed). Errors as rsilu_batch_solve. */
rsilu_status_t rsilu_tune(rsilu_tuner_t t, rsilu_handle_t h, const double *b_dev, double *x_dev,
                          rsilu_tune_result_t *res, hipStream_t s);

/* Solve `count` problems with the autotuner's schedule, on stream s, and wait.
 * Every problem the batched kernel accepts is tuned (rsilu_tune, cached per
 * signature); those the tuner gives to the batched kernel (path 0) start on one
 * batched launch, which lasts as long as its slowest problem, and the plain path
 * (rsilu_solve, one problem after another on a second stream of the batch object,
 * beside the launch) takes the rest. The slowest batched problem moves to the plain path while that shortens
 * the estimated makespan max(slowest batched time, sum of plain times), per
 * iteration (equal iteration counts assumed). The launch uses the tuned tile of
 * its slowest problem (*tile_used, may be NULL). Problems the batched kernel does
 * not accept go to the plain path. path[i] receives 0 (batched) or 1 (plain),
 * res[i] the outcome (status as rsilu_solve). Arguments and errors as
 * rsilu_batch_solve (handles need not be configured for the batched kernel);
 * a plain solve's runtime error is returned after all problems ran. */
rsilu_status_t rsilu_batch_solve_auto(rsilu_batch_t bt, rsilu_tuner_t t, int32_t count, const rsilu_handle_t *hs,
                                      const double *const *b, const double *tol, double *const *x,
                                      rsilu_batch_result_t *res, int32_t *path, rsilu_tile_t *tile_used,
                                      hipStream_t s);

/* Number of cached signatures. */
int32_t rsilu_tuner_size(rsilu_tuner_t t);

void rsilu_tuner_destroy(rsilu_tuner_t t);

#ifdef __cplusplus
}
#endif

#endif /* RSILU_BATCH_H */
