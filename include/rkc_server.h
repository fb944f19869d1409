/*
 * rkc_server.h - C ABI of the integration server built on rkc_integrate.
 *
 * In a reactive-flow code every chemistry call integrates a batch of
 * independent cells over one global step (Niemeyer & Sung, Sec. 2.2 and
 * Sec. 3: the integrator takes initial conditions and a global time step).
 * The server accepts such batches as requests from any number of host
 * threads and runs them on one GPU:
 *   - admission by device-memory footprint: each request needs
 *     footprint = 2 a(8 n) + a(8 n n_species) + a(4 n) bytes (a() rounds up
 *     to 256) of a fixed device arena of opts.budget_bytes; requests wait in
 *     arrival order while the arena or every launch slot is busy;
 *   - batching: the oldest waiting request is launched together with later
 *     waiting requests of the same mechanism, dt, rtol, atol and method, as
 *     one launch of up to opts.max_batch_cells cells (results per cell do not
 *     depend on the batch: rkc_integrate's results depend only on the cell);
 *   - opts.n_streams launches in flight at once, each on its own stream with
 *     its own scratch;
 *   - per-request completion, and latency statistics from submission to
 *     completion.
 * Host arrays are staged through a pinned host mirror of the arena, so
 * callers may pass ordinary (pageable) memory.
 *
 * Conventions as in rkc.h: RKC_OK or a negative RKC_E* code, nothing thrown
 * across the ABI; all functions are thread-safe for one server.
 */
#ifndef RKC_SERVER_H
#define RKC_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "rkc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rkc_server rkc_server;   /* opaque, owned by the library */

typedef struct {
    size_t  budget_bytes;     /* device arena for request state (and the same size of
                                 pinned host memory); default 1 GiB */
    int32_t n_streams;        /* launches in flight, 1..16; default 4 */
    int32_t max_batch_cells;  /* cells per merged launch; default 1048576 */
    int32_t lanes_per_cell;   /* as rkc_opts.lanes_per_cell; default 0 (automatic) */
    int32_t param_placement;  /* as rkc_opts.param_placement; default RKC_PARAMS_AUTO */
} rkc_server_opts;

typedef struct {
    int64_t submitted, completed, failed_requests;  /* failed: an error or a failed cell */
    int64_t launches, cells;                          /* merged launches and their cells */
    int64_t n_rhs;                                    /* source-term evaluations of the cells */
    int64_t peak_bytes, peak_queue;                   /* arena high-water mark, longest queue */
    double  mean_ms, p50_ms, p99_ms, max_ms;          /* submit-to-completion latency of the
                                                         completed requests (nearest rank) */
} rkc_server_stats;

/* Fill *opts with the defaults.  RKC_EINVAL for NULL. */
int rkc_server_opts_default(rkc_server_opts *opts);

/* Create a server on the current HIP device: allocates the arena, its pinned
 * mirror, the streams and starts the dispatcher thread.  opts may be NULL.
 * RKC_EINVAL (n_streams outside 1..16, budget below 1 MiB, max_batch_cells < 1),
 * RKC_ENOMEM, RKC_EDEVICE. */
int rkc_server_create(const rkc_server_opts *opts, rkc_server **out);

/* Wait for every submitted request, stop the dispatcher and free everything
 * (registered mechanisms included).  NULL is accepted. */
int rkc_server_destroy(rkc_server *srv);

/* Create a mechanism owned by the server (same description and errors as
 * rkc_mech_create) and return its id for rkc_server_submit. */
int rkc_server_register_mech(rkc_server *srv, const rkc_mech_desc *desc, int32_t *mech_id);

/* Queue one request: integrate n_cells cells over [0, dt] as rkc_integrate
 * does (T [n] and Y [n][n_species] in/out, P [n]; method RKC_METHOD_*), with
 * the default s_max and max_steps.  The host arrays (and cell_status [n], which
 * may be NULL) must stay valid and untouched until the request completes.
 * *req_id identifies the request.  Errors: RKC_EINVAL (bad id or arguments),
 * RKC_ENOMEM (footprint larger than the whole arena); n_cells = 0 completes
 * at once. */
int rkc_server_submit(rkc_server *srv, int32_t mech_id, size_t n_cells, double *T,
                      const double *P, double *Y, double dt, double rtol, double atol,
                      int32_t method, int32_t *cell_status, uint64_t *req_id);

/* *done = 1 once the request's results are in its arrays, else 0.
 * RKC_EINVAL for an unknown (or already waited-for) id. */
int rkc_server_poll(rkc_server *srv, uint64_t req_id, int32_t *done);

/* Block until the request completes and release its record.  *n_failed (may
 * be NULL) receives the number of cells whose status is not RKC_CELL_OK.
 * Returns RKC_OK, RKC_ECELLS (some cell failed), a device error code, or
 * RKC_EINVAL for an unknown id. */
int rkc_server_wait(rkc_server *srv, uint64_t req_id, int32_t *n_failed);

/* Counters and latency statistics since creation or the last reset. */
int rkc_server_get_stats(rkc_server *srv, rkc_server_stats *stats);
int rkc_server_reset_stats(rkc_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* RKC_SERVER_H */
