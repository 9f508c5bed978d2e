/*
 * spkadd_batch.h -- batched SpKAdd: many independent sums B_r = A_r,1 + ... + A_r,k_r
 * (Section II-A, per request) in one fused sequence of launches, with no host wait
 * between the passes.
 *
 * Each request is an ordinary SpKAdd on CSC inputs (same formats as spkadd.h).  A
 * run enqueues, on one stream: the upload of the request table, the upper bounds
 * and bins of every request's columns (Section III-A), the symbolic pass
 * (Algorithm 6), one exclusive scan per request, and the numeric pass (Algorithm
 * 5) -- all as persistent kernels over one global worklist of columns, so a run
 * costs the same handful of launches however many requests it holds (seven kernels
 * and one copy: by default each pass is one launch over every wavefront bin, see
 * spkadd_opts.batch_fused_cols).  The launch sequence is captured once as a hipGraph
 * per launch shape and replayed.
 *
 * Outputs go to caller buffers sized by an upper bound: cap_c >= sum_i nnz(A_r,i)
 * always suffices (nnz(B) never exceeds it).  The host learns nnz(B_r) only from
 * spkadd_batch_results, after the run.
 *
 * Limits: k_r <= 64.  A column with u_j up to opts.batch_wave_max (1024 by default)
 * runs one wavefront per column; a longer one, up to opts.batch_wg_max (4096 by
 * default), one workgroup per column if its request has at most 2^17 rows.  A
 * request with a longer column is reported as SPKADD_REQ_TOO_LARGE and left for the
 * one-request path (spkadd_plan / spkadd_symbolic / spkadd_numeric).  These cutoffs,
 * the workgroup size, the accumulator choice, the fused launch and the run size are
 * what spkadd_tune_batch (spkadd_tune.h) measures.
 *
 * Memory: requests are HOST structs holding DEVICE pointers (all non-NULL, also for
 * inputs without entries); the batch copies them at run time.  Inputs and outputs
 * must stay valid until the run has finished on the stream.  The batch owns its
 * workspace, sized at creation.
 * Errors: status codes as in spkadd.h; per-request outcomes in spkadd_batch_results.
 * One batch object must not be used by two threads at once.
 */
#ifndef SPKADD_BATCH_H
#define SPKADD_BATCH_H

#include "spkadd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spkadd_request {
  int32_t m, n, k;               /* shape and number of inputs, 1 <= k <= 64 */
  const int32_t* const* colptr;  /* HOST array of k DEVICE pointers, each int32[n+1] */
  const int32_t* const* rowidx;  /* HOST array of k DEVICE pointers */
  const void* const* values;     /* HOST array of k DEVICE pointers (the batch's dtype) */
  int32_t* colptr_c;             /* DEVICE int32[n+1]: colptr(B) */
  int32_t* rowidx_c;             /* DEVICE int32[cap_c] */
  void* values_c;                /* DEVICE float[cap_c] or double[cap_c] */
  int64_t cap_c;                 /* output capacity in entries */
} spkadd_request;

/* per-request outcome (spkadd_batch_results) */
#define SPKADD_REQ_OK 0
#define SPKADD_REQ_TOO_LARGE 1 /* some column has more input entries than a batched run takes
                                  (opts.batch_wg_max, 4096 by default; opts.batch_wave_max, 1024,
                                  in requests of more than 2^17 rows): nothing written */
#define SPKADD_REQ_CAPACITY 2  /* nnz(B) > cap_c: colptr(B) written, rows and values not */

typedef struct spkadd_batch_s* spkadd_batch_t;

/*
 * spkadd_batch_create -- a batch for up to max_requests requests per run, with at
 * most max_columns columns and max_inputs inputs (sum of k) over one run.
 *   dtype : value type of every request.
 *   opts  : NULL for defaults; accum_mode, bitmap_ratio and batch_fused_cols apply
 *           (force_bin, windows and load factors do not).
 * Errors: INVALID, OOM, HIP; UNSUPPORTED for SPKADD_FLAG_ORDERED (the ordered sum
 * runs through spkadd_plan / spkadd_symbolic / spkadd_numeric only).
 */
spkadd_status spkadd_batch_create(spkadd_batch_t* out, spkadd_dtype dtype, int32_t max_requests,
                                  int64_t max_columns, int64_t max_inputs, const spkadd_opts* opts);

/*
 * spkadd_batch_run -- enqueue one run over reqs[0..nreq) on stream.  No host wait,
 * except for the previous run's request-table upload if it is still in flight.
 * use_graph: 1 = launch through the captured hipGraph of this launch shape (captured
 * on first use), 0 = plain launches.
 * Errors: INVALID (bad request fields, more requests / columns / inputs than the
 * batch was created for), HIP.
 */
spkadd_status spkadd_batch_run(spkadd_batch_t b, const spkadd_request* reqs, int32_t nreq, int32_t use_graph,
                               hipStream_t stream);

/*
 * spkadd_batch_results -- wait for the last run and copy nnz(B_r) and the outcome of
 * every request of it into HOST arrays of nreq entries (either may be NULL).
 * Errors: HIP; STATE before any run.
 */
spkadd_status spkadd_batch_results(spkadd_batch_t b, int64_t* nnz, int32_t* status);

/* 1 when the last run has finished on the device (or there was none), 0 while it
 * runs.  Does not wait. */
int32_t spkadd_batch_ready(spkadd_batch_t b);

/* Launch statistics.  A run's launch shape is the set of (wave bin, accumulator)
 * launches its columns can need and its largest bitmap; a run through the graph uses a
 * graph captured for its own shape or, if there is none, for a shape that covers it
 * (its extra launches find no columns and exit), and captures its own shape only when
 * no captured one covers it. */
typedef struct spkadd_batch_info {
  int32_t graphs_captured; /* distinct launch shapes captured so far */
  int32_t graph_replays;   /* runs launched through a captured graph */
  int32_t kernels_per_run; /* kernels in the last captured or plainly launched sequence */
  int32_t graph_reuses;    /* replays of a graph captured for a covering shape */
  int32_t fused_runs;      /* runs whose passes were one launch each (opts.batch_fused_cols) */
  int32_t reserved;
} spkadd_batch_info;
spkadd_status spkadd_batch_get_info(spkadd_batch_t b, spkadd_batch_info* out);

spkadd_status spkadd_batch_destroy(spkadd_batch_t b);

#ifdef __cplusplus
}
#endif
#endif /* SPKADD_BATCH_H */
