/*
 * spkadd.h -- C ABI of the MI355X (gfx950) SpKAdd library.
 *
 * SpKAdd (Section II-A of "Parallel Algorithms for Adding a Collection of Sparse
 * Matrices") computes B = A_1 + A_2 + ... + A_k for k sparse matrices that all have
 * the same shape m x n.  This library implements the paper's hash and sliding-hash
 * k-way method (Algorithms 5-8) as GPU kernels:
 *   plan     -- upper bound u_j = sum_i nnz(A_i(:,j)) per column, binning of the
 *               columns, and the row windows used for columns too large for one
 *               on-chip table (the sliding hash, Section III-B);
 *   symbolic -- nnz(B(:,j)) per column with a key-only hash table (Algorithm 6,
 *               Section II-D), then an exclusive scan that gives colptr(B);
 *   numeric  -- per-column hash accumulation (Algorithm 5), then an in-LDS sort of
 *               each output column and a coalesced write of rows and values.
 *
 * Formats (Section II-A, CSC storage).  Every matrix is CSC with
 *   colptr : int32[n+1], colptr[0] = 0, non-decreasing;
 *   rowidx : int32[nnz], rows in [0, m), strictly ascending within each column (in any
 *            order under SPKADD_FLAG_UNSORTED_IN);
 *   values : float[nnz] (SPKADD_F32) or double[nnz] (SPKADD_F64).
 * The output B is canonical CSC in the same form.  Its pattern is the union of
 * the input patterns: explicit zeros and cancellations stay stored, because the
 * paper's accumulators never test values.  Its rows are ascending.
 *
 * Memory.  Every array argument documented as DEVICE is GPU memory on the current
 * HIP device.  Every "array of pointers" argument is HOST memory that holds k
 * DEVICE pointers; it is read during the call and not kept.  The caller owns all
 * inputs and outputs.  The plan owns its workspace, which comes from a
 * stream-ordered cache inside the library.  Inputs must stay unchanged and alive
 * from spkadd_plan until spkadd_numeric has finished on the stream.
 *
 * Errors.  Every call returns a status and throws no exceptions.  spkadd_last_error()
 * gives a message for the calling thread.  On an error, outputs are unspecified.
 * The plan, symbolic and numeric calls clear the HIP runtime's last-error state of
 * the calling thread on entry (so that a stale status of the caller's own earlier
 * HIP calls is not taken for a failure of theirs).
 * The plan stays usable unless the status is SPKADD_ERR_HIP, which marks it failed.
 * Argument checks run on the host before any device work.
 *
 * Threads.  Different plans may be used from different threads.  One plan must
 * not be used by two threads at once.
 */
#ifndef SPKADD_H
#define SPKADD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spkadd_status {
  SPKADD_OK = 0,
  SPKADD_ERR_INVALID = 1,     /* bad argument, or malformed input found by validation */
  SPKADD_ERR_OOM = 2,         /* device or host allocation failed */
  SPKADD_ERR_HIP = 3,         /* a HIP runtime call failed; the plan is unusable */
  SPKADD_ERR_STATE = 4,       /* calls out of order (numeric before symbolic) */
  SPKADD_ERR_OVERFLOW = 5,    /* a count does not fit int32 (u_j, nnz(B)) */
  SPKADD_ERR_UNSUPPORTED = 6  /* a size the library does not handle (see spkadd_plan) */
} spkadd_status;

typedef enum spkadd_dtype { SPKADD_F32 = 0, SPKADD_F64 = 1 } spkadd_dtype;

/* opts.flags */
#define SPKADD_FLAG_VALIDATE 1u /* check every input on the device in spkadd_plan */
#define SPKADD_FLAG_TRACE 2u    /* time every kernel launch with HIP events */
#define SPKADD_FLAG_TRACE_NUMERIC 4u /* time only the launches of spkadd_numeric */
#define SPKADD_FLAG_UNSORTED_OUT 8u  /* the rows of each output column may come in any order: the hash
                                        accumulators skip their sort (the paper's "if sorted output is
                                        desired", Algorithm 5); bitmap accumulators are sorted anyway */
#define SPKADD_FLAG_UNSORTED_IN 16u  /* the rows of each input column may come in any order (hash
                                        accumulation needs none, Table I).  The row windows of long
                                        columns then count their entries by histogram and partition
                                        them into one bucket per window in spkadd_plan (about 16 bytes
                                        of device memory per such entry, plus 4 or 8 gathered in
                                        each spkadd_numeric) instead of binary-searching sorted
                                        columns.  Duplicate rows within a column are still summed. */
#define SPKADD_FLAG_ORDERED 32u      /* every value of B is the sequential sum of its terms in input
                                        order i = 1..k, one rounding per addition in the values' type
                                        (the order in which Algorithm 5 visits the inputs of a column,
                                        Section II-C): c = a_first, then c = c + a for each later term.
                                        Results are then reproducible bit for bit, whatever the launch.
                                        spkadd_numeric runs one more pass that re-reads the inputs and
                                        rewrites the values.  The output is sorted (UNSORTED_OUT is
                                        ignored).  With SPKADD_FLAG_UNSORTED_IN, spkadd_plan returns
                                        SPKADD_ERR_UNSUPPORTED; so it does when k is so large that the
                                        pass's per-unit table of the k inputs does not fit on chip
                                        (k above about 2700). */

/* opts.force_bin: test hook that routes columns to one accumulator family */
#define SPKADD_BIN_AUTO (-1)
#define SPKADD_BIN_WAVE 0   /* one wavefront per column (columns with u_j <= 1024) */
#define SPKADD_BIN_WG 1     /* one workgroup per column (columns with u_j <= window_cap) */
#define SPKADD_BIN_WINDOW 2 /* sliding-hash row windows for every non-empty column */

/* opts.accum_mode */
#define SPKADD_ACCUM_AUTO 0
#define SPKADD_ACCUM_HASH 1
#define SPKADD_ACCUM_BITMAP 2

/* Tuning and test options.  Zero-initialised fields (or opts == NULL) mean "auto". */
typedef struct spkadd_opts {
  uint32_t flags;        /* SPKADD_FLAG_* */
  int32_t force_bin;     /* SPKADD_BIN_*; 0 is "wave", so use SPKADD_BIN_AUTO (-1) for auto */
  int32_t window_cap;    /* max input entries per row window and per workgroup column;
                            0 = auto.  Small values force the sliding hash on small inputs. */
  int32_t hash_mode;     /* 0 = multiplicative hash; 1 = degenerate hash (every row starts
                            probing at slot 0), a test hook for long probe chains */
  int32_t wave_max;      /* largest u_j handled one wavefront per column (64..1024); 0 = auto */
  float load_factor_sym; /* max (input entries / table slots) of symbolic tables; 0 = auto */
  float load_factor_num; /* max (output entries / table slots) of numeric tables, <= 0.5; 0 = auto */
  float window_fill;     /* target fill of a row window relative to window_cap; 0 = auto */
  int32_t accum_mode;    /* wave bins: 0 = auto (bitmap where dense enough, else hash),
                            1 = hash tables only, 2 = bitmap wherever it fits (m <= 131072) */
  float bitmap_ratio;    /* auto mode: use the bitmap when ceil(m / 8192) <= bitmap_ratio * E,
                            E = ceil(u_max / 64) of the bin; 0 = default (1.0) */
  int32_t wave_merge;    /* 0 = merge two adjacent wave bins that each hold >= 1/16 of the
                            wave columns (one kernel then reads neighbouring columns together);
                            1 = keep every wave bin separate */
  int32_t batch_fused_cols; /* batched runs (spkadd_batch.h): a run with at most this many
                              columns in total does each pass in one launch over every wave
                              bin; larger runs launch one kernel per bin and accumulator.
                              0 = default (no limit: every run), negative = never */
  int32_t batch_wave_max;   /* batched runs: a column with u_j up to this goes one wavefront per
                              column (64..1024; 0 = 1024) */
  int32_t batch_wg_max;     /* batched runs: longer columns with up to this many entries go one
                              workgroup per column (requests of at most 2^17 rows); longer ones
                              make the request SPKADD_REQ_TOO_LARGE (batch_wave_max..4096;
                              0 = 4096) */
  int32_t batch_wg_threads; /* batched runs: threads of those workgroups, 256 or 512 (0 = 256) */
  int32_t batch_run_size;   /* requests per batched run found fastest by spkadd_tune_batch; the
                              serving loop uses it when its config's max_batch is 0 (0 = none) */
} spkadd_opts;

typedef struct spkadd_plan_s* spkadd_plan_t;

/* Writes the defaults into *opts (force_bin = SPKADD_BIN_AUTO, everything else auto). */
void spkadd_opts_default(spkadd_opts* opts);

/*
 * spkadd_plan -- set up B = A_1 + ... + A_k (Section II-A) and run the planning step:
 * the per-column upper bounds u_j = sum_i nnz(A_i(:,j)), the binning of the columns
 * (the load balance of Section III-A), and the row windows of the columns that take
 * the sliding hash (Section III-B).
 *   out    : receives the plan (HOST pointer).
 *   m, n   : rows and columns of every matrix, 0 <= m, n <= INT32_MAX - 1.
 *   k      : number of inputs, k >= 1.
 *   colptr : HOST array of k DEVICE pointers, each int32[n+1].
 *   rowidx : HOST array of k DEVICE pointers, each int32[colptr_i[n]].
 *   dtype  : value type of the later spkadd_numeric calls.
 *   opts   : NULL for defaults.
 *   stream : HIP stream for all device work.  The call normally returns without
 *            waiting for the device: the bin counts are copied back asynchronously,
 *            and spkadd_symbolic (or spkadd_get_stats) waits for them after it has
 *            launched the symbolic pass of the columns binned for one wavefront,
 *            which reads the bins on the device.  The row windows are then built in
 *            that call.  The plan waits here instead (once for the bin counts, a
 *            few more times for row windows) when SPKADD_FLAG_VALIDATE is set, when
 *            some rowidx pointer is NULL, and when k > 64 or load_factor_num is not
 *            0.5 (the wave bins then take one launch each).
 * Errors: INVALID (null pointers, k < 1, negative sizes, bad option values, or
 * malformed inputs when SPKADD_FLAG_VALIDATE is set), OOM, HIP; OVERFLOW (some u_j
 * above INT32_MAX) here when the plan waits, else from spkadd_symbolic.
 */
spkadd_status spkadd_plan(spkadd_plan_t* out, int32_t m, int32_t n, int32_t k, const int32_t* const* colptr,
                          const int32_t* const* rowidx, spkadd_dtype dtype, const spkadd_opts* opts,
                          hipStream_t stream);

/*
 * spkadd_symbolic -- nnz(B(:,j)) for every column with a key-only hash table per
 * column or row window (Algorithms 6 and 7, Section II-D), then colptr(B) by an
 * exclusive scan.
 *   colptr_c : DEVICE int32[n+1], written with colptr(B).  It must stay valid until
 *              spkadd_numeric has finished, which reads it.
 *   nnz_c    : HOST int64 receiving nnz(B).  This call waits on the stream.  When
 *              the plan's stream differs, the first call orders itself after the
 *              plan's device work.
 * Errors: INVALID (null arguments), OVERFLOW (nnz(B) > INT32_MAX, or some u_j above
 * INT32_MAX when spkadd_plan did not wait), UNSUPPORTED (row windows that need more
 * LDS than the device has, when spkadd_plan did not wait), HIP.
 * It may be called again; every call recomputes the counts.
 */
spkadd_status spkadd_symbolic(spkadd_plan_t plan, int32_t* colptr_c, int64_t* nnz_c, hipStream_t stream);

/*
 * spkadd_numeric -- the values of B (Algorithms 5 and 8): each column or row window
 * is accumulated in an on-chip hash table.  Its entries are then sorted by row on
 * chip and written to rowidx_c / values_c at colptr(B).
 *   values   : HOST array of k DEVICE pointers to the input values (float or double
 *              as the plan's dtype), aligned with the rowidx arrays given to spkadd_plan.
 *              Every pointer must be non-NULL unless all inputs are empty; the pointer
 *              of an input without entries is never read through.
 *   rowidx_c : DEVICE int32[nnz(B)].
 *   values_c : DEVICE float[nnz(B)] or double[nnz(B)].
 * The call is asynchronous on `stream`.  It may be repeated with new values for
 * the same patterns.
 * Errors: STATE (spkadd_symbolic not yet run), INVALID (NULL arguments), HIP.
 */
spkadd_status spkadd_numeric(spkadd_plan_t plan, const void* const* values, int32_t* rowidx_c, void* values_c,
                             hipStream_t stream);

/*
 * spkadd_sum_noalloc -- B = A_1 + ... + A_k in one call (spkadd_plan, spkadd_symbolic
 * and spkadd_numeric in turn) that allocates nothing: for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that must not
 * allocate, harnesses that forbid hipMalloc).  Every byte of device workspace comes
 * from one static array of SPKADD_NOALLOC_SCRATCH_BYTES per GPU, held by the library
 * from first use until the process ends; summaries come back through pageable host
 * memory after a wait on the stream.  No hipMalloc, hipFree, pinned allocation or
 * event creation happens inside the call.
 *   m, n, k, colptr, rowidx, dtype, opts : as spkadd_plan (trace flags are ignored).
 *   values   : as spkadd_numeric.
 *   colptr_c : DEVICE int32[n+1], written with colptr(B).
 *   rowidx_c, values_c : DEVICE arrays of cap_c entries.
 *   cap_c    : capacity of rowidx_c / values_c in entries.
 *   nnz_c    : HOST int64 receiving nnz(B).
 * The call waits on the stream a few times (as spkadd_plan and spkadd_symbolic do);
 * the numeric pass is still running on the stream when it returns.
 * The scratch array is shared by every call on a GPU and keeps the last call's
 * contents (the library clears what it needs): calls on one GPU must be ordered
 * (one stream, or synchronised) -- calls that overlap on one GPU race.
 * Errors: as spkadd_plan / spkadd_symbolic / spkadd_numeric; UNSUPPORTED when the
 * inputs need more workspace than the array holds (about 18 bytes per column plus
 * 24 per input, and, when some column needs row windows, about 8 k + 64 bytes per
 * window and 4 k + 40 per window of each refinement level: with 64 MiB, n up to
 * about 3.5 million columns without windows); INVALID when nnz(B) > cap_c
 * (colptr_c and *nnz_c are then written,
 * rowidx_c and values_c are not).
 */
#define SPKADD_NOALLOC_SCRATCH_BYTES (64u << 20)
spkadd_status spkadd_sum_noalloc(int32_t m, int32_t n, int32_t k, const int32_t* const* colptr,
                                 const int32_t* const* rowidx, const void* const* values, spkadd_dtype dtype,
                                 const spkadd_opts* opts, int32_t* colptr_c, int32_t* rowidx_c, void* values_c,
                                 int64_t cap_c, int64_t* nnz_c, hipStream_t stream);

/* spkadd_free -- return the plan's workspace to the library cache and release the
 * plan.  The workspace is reused only after the work queued on the plan's last
 * stream is done.  NULL is a no-op. */
spkadd_status spkadd_free(spkadd_plan_t plan);

/* Message describing the last error on the calling thread ("" if none).  It stays
 * valid until the next call from the same thread. */
const char* spkadd_last_error(void);

/* Per-plan statistics, filled after spkadd_plan (a plan that has not waited for its
 * bin counts waits here); nnz_out after spkadd_symbolic. */
typedef struct spkadd_stats {
  int64_t nnz_in;        /* sum_i nnz(A_i) */
  int64_t nnz_out;       /* nnz(B), -1 before spkadd_symbolic */
  int32_t n_empty_cols;  /* columns with u_j = 0 */
  int32_t n_wave_cols;   /* columns handled one wavefront each */
  int32_t n_wg_cols;     /* columns handled one workgroup each */
  int32_t n_window_cols; /* columns split into row windows (sliding hash) */
  int32_t n_windows;     /* row windows over all window columns */
  int32_t window_levels; /* refinement rounds the window split needed */
  int32_t window_cap;    /* input entries per window target used */
  int32_t wave_max;      /* wave bin limit used */
} spkadd_stats;
spkadd_status spkadd_get_stats(spkadd_plan_t plan, spkadd_stats* out);

/* Kernel timings recorded under SPKADD_FLAG_TRACE (or SPKADD_FLAG_TRACE_NUMERIC) by the
 * last plan / symbolic / numeric calls of this plan.  spkadd_trace_count gives how many launches were
 * recorded.  spkadd_trace_get copies the kernel name of launch idx (NUL-terminated,
 * at most name_cap bytes) and its elapsed milliseconds.  It waits for the events to
 * complete. */
int32_t spkadd_trace_count(spkadd_plan_t plan);
spkadd_status spkadd_trace_get(spkadd_plan_t plan, int32_t idx, char* name, int32_t name_cap, float* ms);
/* Clears the recorded launches of the plan. */
spkadd_status spkadd_trace_reset(spkadd_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* SPKADD_H */
