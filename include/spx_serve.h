/*
 * spx_serve.h -- serving loop over resident sparse matrices (part of libspx).
 *
 * The paper's break-even argument (Section 7) is that a format's conversion pays off over many
 * products with the same matrix.  A server makes that the normal case: matrices are converted
 * once, kept resident in device memory, and products are requested against them.  Requests for
 * one matrix that are waiting at the same time are coalesced into one product with several
 * right-hand sides (spx_spmm), so the matrix stream is read once for the whole batch.
 *
 * Model:
 *   - A server owns a memory budget.  spx_server_add_matrix admits a matrix only if an upper
 *     bound of its footprint, together with the slots' staging bound, fits in what is left
 *     (otherwise SPX_ERR_NOMEM and nothing is converted); removing a matrix returns its bytes.
 *     The staging bound is slots x the largest per-batch staging (x and y columns, hot rows, tile
 *     carries for max_batch requests) of any matrix admitted so far; it is never released.
 *   - A request names a resident matrix, an input x (n floats) and an output y (m floats), both
 *     caller-owned device memory that must stay valid until the request completes, and the
 *     stream whose work produces x: the request's product waits (on the device) for the work
 *     enqueued on that stream before the submission.  With a NULL stream the caller guarantees
 *     that x is complete when it submits.
 *       SPX_REQ_SPMV:      y = A x
 *       SPX_REQ_PAGERANK:  y = d A x + (1 - d) / n   (one power-iteration step with damping d on a
 *                          column-stochastic A; the caller supplies the normalised matrix)
 *   - A scheduler thread owns all device work after admission.  It keeps up to `slots` batches in
 *     flight, each on its own stream with its own product scratch.  Whenever a slot is free it
 *     takes the matrix whose oldest waiting request is oldest, coalesces up to max_batch of that
 *     matrix's waiting requests (oldest first) and launches them as one product; a popular matrix
 *     may have batches on several slots at once.  Requests that arrive while batches run are
 *     admitted as slots free up (continuous batching).
 *   - With coalesce = 0 the server is the plain path: one slot, one request per launch, in arrival
 *     order, through the single-vector product.
 *   - Each column of a batched product is the same computation as the request alone up to the
 *     summation order inside a tile, so results agree with the request served alone within the
 *     FP32 dot-product error bound (integer-valued inputs: exactly).
 *
 * Matrices must be CRS (row-split or merge) stored in FP32 or bfloat16 (x and y are FP32).
 * Thread safety: submit / wait / stats may be called from any thread; add / remove / destroy from
 * one thread at a time.
 */
#ifndef SPX_SERVE_H
#define SPX_SERVE_H

#include "spx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spx_server_s* spx_server;

typedef struct {
    int64_t memory_budget; /* bytes for resident matrices (> 0)                        */
    int32_t slots;         /* batches in flight at once, one stream each (1 .. 16)      */
    int32_t max_batch;     /* requests coalesced into one product (1 .. 64)             */
    int32_t coalesce;      /* 1: coalesce waiting requests; 0: plain path (see above)    */
    int32_t poll_us;       /* scheduler's sleep between completion checks (0 .. 1000)   */
} spx_server_opts;

#define SPX_REQ_SPMV 0
#define SPX_REQ_PAGERANK 1

typedef struct {
    int32_t matrix;  /* id from spx_server_add_matrix                         */
    int32_t kind;    /* SPX_REQ_SPMV or SPX_REQ_PAGERANK                       */
    float damping;   /* d of SPX_REQ_PAGERANK, in [0, 1]; ignored for SPMV     */
    const float* x;  /* device, n floats                                       */
    float* y;        /* device, m floats, must not overlap x                   */
    void* stream;    /* hipStream_t producing x (the product waits for it), or NULL
                      * when x is already complete                              */
} spx_request;

typedef struct {
    int64_t requests;        /* completed                                              */
    int64_t batches;         /* launches                                               */
    int64_t max_batch_seen;  /* widest batch launched                                  */
    int64_t bytes_resident;  /* footprint bounds of the admitted matrices              */
    int64_t memory_budget;
    int32_t matrices;        /* resident                                               */
    int32_t in_flight;       /* batches on the device now                              */
    int64_t bytes_staging;   /* staging bound reserved for the slots (within the budget) */
} spx_server_stats;

/* Defaults: budget 64 GiB, 4 slots, max_batch 32, coalesce 1, poll_us 0 (the scheduler yields
 * instead of sleeping while batches are in flight). */
spx_status spx_server_opts_default(spx_server_opts* opts);

/* Create a server (starts its scheduler thread and streams on the current device). */
spx_status spx_server_create(const spx_server_opts* opts, spx_server* out);

/* Wait for every submitted request, stop the scheduler, free all resident matrices. */
spx_status spx_server_destroy(spx_server S);

/*
 * Convert triplets (as spx_convert) and keep the result resident.  fmt: SPX_CSR_ROWSPLIT or
 * SPX_CSR_MERGE; opts->value_type: SPX_F32 or SPX_BF16 (opts may not be NULL).  Admission: the
 * footprint bound (stored arrays for coo->nnz entries, partition tables, product scratch for
 * max_batch columns) must fit in the budget not yet taken, else SPX_ERR_NOMEM with nothing
 * converted.  *id receives the matrix id; *bytes (nullable) its footprint bound.  Conversion runs
 * on `stream` and is complete when the call returns.
 */
spx_status spx_server_add_matrix(spx_server S, const spx_coo_desc* coo, spx_format fmt,
                                 const spx_convert_opts* opts, void* stream, int32_t* id,
                                 int64_t* bytes);

/* Wait for the matrix's requests, then free it and return its bytes to the budget. */
spx_status spx_server_remove_matrix(spx_server S, int32_t id);

/* Queue one request; *ticket identifies it for spx_server_wait.  When req->stream is not NULL an
 * event is recorded on it here and the product waits for that event.  Errors (INVALID_ARG for an
 * unknown matrix, NULL vectors or a bad kind, ALIAS for overlapping x and y, HIP when the event
 * cannot be recorded) are reported here, before anything is queued. */
spx_status spx_server_submit(spx_server S, const spx_request* req, uint64_t* ticket);

/* Block until the request completes (its y is written and visible to the device) and forget the
 * ticket.  latency_us (nullable): time from submit until the scheduler saw the batch finish. */
spx_status spx_server_wait(spx_server S, uint64_t ticket, double* latency_us);

/*
 * Open-loop load: submit reqs[i] when arrival_us[i] microseconds have passed since the call
 * started (arrival_us ascending; the calling thread spins between arrivals), then wait for all of
 * them.  latency_us[i] receives each request's latency; *wall_us (nullable) the time from the
 * first submission to the last completion.  Stops at the first invalid request (its status is
 * returned; earlier requests still complete).
 */
spx_status spx_server_replay(spx_server S, const spx_request* reqs, const double* arrival_us,
                             int64_t count, double* latency_us, double* wall_us);

spx_status spx_server_get_stats(spx_server S, spx_server_stats* stats);

#ifdef __cplusplus
}
#endif
#endif
