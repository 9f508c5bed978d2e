/*
 * spkadd_server.h -- a serving loop for SpKAdd requests (continuous batching).
 *
 * Clients submit requests (each an SpKAdd, Section II-A) from any thread and wait
 * on tickets.  A server thread admits requests in arrival order while their output
 * memory fits the HBM budget and a stream has room for another run (config depth),
 * groups them into batched runs (include/spkadd_batch.h) over one or more streams,
 * and completes the tickets.  A request that a batch reports as too large
 * (a column with more entries than opts.batch_wg_max, 4096 by default, or than
 * opts.batch_wave_max in a request of more than 2^17 rows) goes through the
 * one-request path (spkadd_plan / spkadd_symbolic / spkadd_numeric) on one of the
 * one-request lanes (config large_streams), each with a stream of its own.  Requests that arrive while others are on the device join the next run.
 *
 * Outputs are allocated by the server (stream-ordered, or reused from released
 * tickets) with the capacity the request states in cap_c (sum_i nnz(A_i) always
 * suffices) and stay owned by the server until spkadd_server_release.  Held and kept
 * output memory together stay within the HBM budget.  Inputs must stay valid until
 * the ticket completes.
 *
 * While runs are in flight, and for 0.5 ms after its last work, the server thread
 * polls every few microseconds (one host core busy); idle longer, it sleeps until a
 * submit.  spkadd_server_wait polls its ticket for up to 2 ms before it sleeps.
 */
#ifndef SPKADD_SERVER_H
#define SPKADD_SERVER_H

#include "spkadd_batch.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spkadd_server_s* spkadd_server_t;

typedef struct spkadd_server_config {
  spkadd_dtype dtype;
  int32_t n_streams;       /* streams that batched runs rotate over (1..8) */
  int32_t max_batch;       /* requests per batched run (1..4096); 0 = opts->batch_run_size
                              (the run size spkadd_tune_batch found fastest) if set, else 8 */
  int32_t depth;           /* runs in flight per stream (1 or 2): with 1, requests that
                              arrive while a stream's run executes wait and join its
                              next run (larger runs); with 2, the next run is enqueued
                              behind the running one */
  int32_t large_streams;   /* one-request lanes (0..8; 0 = 2): requests too large for a
                              batched run are served on this many streams at once, each
                              lane a host thread with its own stream */
  int64_t max_columns;     /* columns per batched run */
  int64_t max_inputs;      /* inputs (sum of k) per batched run */
  uint64_t hbm_budget;     /* bytes of output memory the admitted requests may hold */
  const spkadd_opts* opts; /* NULL for defaults */
} spkadd_server_config;

#define SPKADD_REQ_ERROR 3 /* the run failed: see spkadd_result.error */

typedef struct spkadd_result {
  int32_t status;          /* SPKADD_REQ_OK, SPKADD_REQ_CAPACITY or SPKADD_REQ_ERROR */
  int32_t error;           /* spkadd_status of a failed run, SPKADD_OK otherwise */
  int32_t path;            /* 0 = batched run, 1 = one-request path */
  int32_t reserved;
  int64_t nnz;             /* nnz(B) */
  int32_t* colptr_c;       /* DEVICE, owned by the server until release */
  int32_t* rowidx_c;
  void* values_c;
  double t_submit, t_start, t_done; /* seconds on the server's steady clock */
} spkadd_result;

/* Starts the server thread.  Errors: INVALID, OOM, HIP. */
spkadd_status spkadd_server_create(spkadd_server_t* out, const spkadd_server_config* cfg);

/* Queues a request (a HOST struct; its pointer arrays are copied, its output fields are
 * ignored).  The request's output memory must fit the budget on its own.
 * Errors: INVALID (bad request, k > 64, too large for the budget), STATE (stopping). */
spkadd_status spkadd_server_submit(spkadd_server_t s, const spkadd_request* req, uint64_t* ticket);

/* Waits until the ticket completes (timeout_s < 0: no limit).
 * Errors: INVALID (unknown ticket), STATE (timeout: the ticket is still pending). */
spkadd_status spkadd_server_wait(spkadd_server_t s, uint64_t ticket, spkadd_result* out, double timeout_s);

/* Gives the ticket's outputs back to the server and forgets the ticket.  The server
 * keeps released output blocks for later requests of the same size class (a power of
 * two of at least 64 KiB), so the caller must have finished every use of the outputs,
 * also work it enqueued on its own streams. */
spkadd_status spkadd_server_release(spkadd_server_t s, uint64_t ticket);

/* Current time on the server's clock (seconds), for stamping arrivals. */
double spkadd_server_now(spkadd_server_t s);

typedef struct spkadd_server_info {
  int64_t runs;            /* batched runs launched */
  int64_t batched;         /* requests served by batched runs (including those sent on) */
  int64_t large;           /* requests sent to the one-request path */
  int64_t allocations;     /* output blocks allocated (the rest were reused) */
  uint64_t held_bytes;     /* output memory held by tickets */
  uint64_t pooled_bytes;   /* released output memory kept for reuse */
  int32_t graphs_captured; /* over every batch object of the server */
  int32_t graph_reuses;
} spkadd_server_info;

/* Counters since creation.  Errors: INVALID. */
spkadd_status spkadd_server_get_info(spkadd_server_t s, spkadd_server_info* out);

/* Finishes the runs in flight, cancels the requests not yet admitted (their tickets
 * complete with status SPKADD_ERR_STATE), stops the threads and frees everything,
 * including outputs not yet released. */
spkadd_status spkadd_server_destroy(spkadd_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* SPKADD_SERVER_H */
