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
 * device allocation happens while serving), solved by rsilu_solve on its
 * slot's stream and copied back; then its bytes and its slot return to the
 * pool at once, so requests that arrived meanwhile join while the others are
 * still on the GPU. Solves on different slots overlap on the device (the
 * single-workgroup sweeps of one solve leave almost every compute unit free).
 * The per-request arithmetic is exactly that of a lone rsilu_solve call, so a
 * result does not depend on what else was in flight.
 *
 * All calls are thread-safe. No call throws.
 */
#ifndef RSILU_SERVE_H
#define RSILU_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "rsilu.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsilu_server *rsilu_server_t;

typedef struct {
    int32_t device;        /* HIP device ordinal */
    int32_t slots;         /* solves on the device at once (one stream each), >= 1 */
    int32_t setup_threads; /* host threads running rsilu_factor, >= 1 */
    int32_t reserved;
    size_t hbm_bytes;      /* size of the device arena holding every admitted request */
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
} rsilu_result_t;

/* Start a server: allocates the arena (hbm_bytes) on `device`, creates one
 * stream per slot and starts the threads. EINVAL for bad options, ENOMEM if
 * the arena cannot be allocated, EHIP for other runtime errors. */
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
