/*
 * rsilu serving runtime: a stream of independent least-squares requests
 * (each its own sparse A and b) solved on one GPU with continuous admission.
 *
 * Every request goes through the host setup of rsilu_factor (on one of
 * `setup_threads` host threads) and then waits for admission: it is admitted
 * when a solve slot is free and its device footprint (rsilu_device_bytes plus
 * its b and x) fits in what is left of the server's HBM arena. Admission is
 * first come, first served in order of setup completion. An admitted request
 * is uploaded into the arena (allocated once, at rsilu_server_create; no
 * device allocation happens while serving), solved on its slot's stream and
 * copied back; then its bytes and its slot return to the pool at once, so
 * requests that arrived meanwhile join while the others are still on the GPU.
 *
 * With batch_max = 0 every admitted request is solved alone by rsilu_solve.
 * With batch_max >= 1 a free slot admits, first come first served, up to
 * batch_max ready requests that fit in the arena together. Without the
 * autotuner (tune_slack = 0) those the batched kernel accepts
 * (rsilu_batch_accepts) share one persistent launch with 1024 threads, 4
 * and 4 lanes (rsilu_batch.h), the others take rsilu_solve. With the autotuner
 * (tune_slack > 0) an admission holding at least two accepted requests is
 * scheduled by rsilu_batch_solve_auto (one batched launch, the slowest requests
 * on the plain path beside it), and a lone request takes the plain path
 * untuned, so under light load requests keep the plain path's latency and a
 * burst shares launches. Slots run their launches concurrently, so a launch of
 * new arrivals overlaps the launches already on the device.
 *
 * A result does not depend on what else was in flight: it is bit for bit the
 * result of a lone rsilu_solve (path 1) or of a lone rsilu_batch_solve with
 * the reported tile (path 0). With the autotuner, a problem signature keeps the
 * tile and times of its first tuning for the server's lifetime (tune_slack only
 * enables it: the split needs no slack).
 *
 * All calls are thread-safe. No call throws.
 */
#ifndef RSILU_SERVE_H
#define RSILU_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "rsilu.h"
#include "rsilu_batch.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsilu_server *rsilu_server_t;

typedef struct {
    int32_t device;        /* HIP device ordinal */
    int32_t slots;         /* solves on the device at once (one stream each), >= 1 */
    int32_t setup_threads; /* host threads running rsilu_factor, >= 1 */
    int32_t batch_max;     /* 0: one rsilu_solve per request; >= 1: requests per launch (<= 65535) */
    size_t hbm_bytes;      /* size of the device arena holding every admitted request */
    double tune_slack;     /* > 0: schedule admissions with the autotuner (rsilu_tuner_create
                              with this slack); 0: the batched kernel with 1024 threads, 4 and
                              4 lanes for every request it accepts */
    double batch_wait_ms;  /* batch_max >= 2: after admitting a request, a slot waits up to
                              this long for more requests to finish their setup (while any
                              are in setup and fewer than batch_max are ready), so arrivals
                              close together share a launch; 0: no wait */
} rsilu_server_opts_t;

typedef struct {
    int64_t m, n;             /* A is m x n, m >= n */
    const int64_t *rowptr;    /* host CSR of A (as rsilu_factor); copied by submit */
    const int32_t *colind;
    const double *val;
    const double *b;          /* host, m values; copied by submit */
    double *x;                /* host, n values: written before the request's result is
                                 returned; must stay valid until then */
    double tol;               /* stop when ||A^T r|| <= tol ||A^T b|| */
    rsilu_params_t params;    /* setup and solve parameters of this request */
    void *user;               /* returned unchanged in the result */
} rsilu_request_t;

typedef struct {
    int64_t id;               /* from rsilu_server_submit */
    void *user;
    int32_t status;           /* rsilu_status_t of the setup or of the solve */
    int32_t iters;
    double atr_norm, atr_rel; /* as rsilu_solve */
    double setup_ms;          /* host setup (rsilu_factor) */
    double wait_ms;           /* setup done -> admitted */
    double solve_ms;          /* admitted -> x copied back (upload, solve, copy) */
    double total_ms;          /* submit -> done */
    size_t device_bytes;      /* arena bytes the request held */
    int32_t path;             /* 0: batched persistent kernel, 1: rsilu_solve, -1: not solved */
    int32_t launch_size;      /* requests solved by the same launch (1 on path 1) */
    rsilu_tile_t tile;        /* path 0: the tile of the launch */
} rsilu_result_t;

/* Start a server: allocates the arena (hbm_bytes) on `device`, creates one
 * stream (and, with batch_max >= 1, one batch object) per slot and the
 * autotuner, and starts the threads. EINVAL for bad options (slots or
 * setup_threads < 1, batch_max outside [0, 65535], tune_slack negative or not
 * finite, batch_wait_ms negative or not finite), ENOMEM if the arena cannot be allocated, EHIP for other runtime
 * errors. */
rsilu_status_t rsilu_server_create(const rsilu_server_opts_t *opts, rsilu_server_t *out);

/* Queue one request. Host inputs are copied before the call returns; *id (may
 * be NULL) receives its id (0, 1, 2, ... in submit order). EINVAL for NULL or
 * inconsistent arguments, ESTATE after rsilu_server_destroy began. A request
 * larger than the whole arena completes with status ENOMEM. */
rsilu_status_t rsilu_server_submit(rsilu_server_t s, const rsilu_request_t *req, int64_t *id);

/* Copy up to `max` completed results into out (in completion order) and
 * return how many; waits up to wait_ms milliseconds for the first one
 * (0: do not wait). A result is returned once. */
int32_t rsilu_server_poll(rsilu_server_t s, rsilu_result_t *out, int32_t max, int32_t wait_ms);

/* Wait until every submitted request has completed (results stay queued for
 * rsilu_server_poll). */
rsilu_status_t rsilu_server_drain(rsilu_server_t s);

/* Drain, stop the threads and free the arena, streams and queued results.
 * NULL is ignored. */
void rsilu_server_destroy(rsilu_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* RSILU_SERVE_H */
