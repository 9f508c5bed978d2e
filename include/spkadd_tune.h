/*
 * spkadd_tune.h -- autotuning of the SpKAdd launch parameters, cached per device and
 * shape class.
 *
 * The paper measures the sliding hash against its table size (Section IV, Fig. 4):
 * the best size tracks the size of the cache the tables live in, and it differs
 * between its two machines.  The same holds for the choices here (LDS instead of L1 /
 * last-level cache): which columns a wavefront takes (wave_max), which accumulator a
 * wavefront uses (accum_mode, bitmap_ratio), whether neighbouring wavefront bins share
 * a launch (wave_merge), the table load factor (load_factor_sym) and, for the columns
 * too long for one workgroup table, the row-window capacity and fill (window_cap,
 * window_fill) -- the last is Fig. 4's parameter.  spkadd_tune measures them on the
 * caller's own inputs and keeps the fastest setting in a process-wide cache under
 * the input's shape class; spkadd_tune_lookup applies a cached setting to the opts of
 * a later spkadd_plan.  The cache can be saved to and loaded from a JSON file.
 *
 * Search: coordinate descent from the caller's opts (or the defaults) -- every value
 * of one parameter with the others fixed, keep the fastest, next parameter.  The
 * window parameters are searched only when some column is too long for a wavefront.
 * A trial is the whole call sequence spkadd_plan / spkadd_symbolic / spkadd_numeric /
 * spkadd_free with a stream synchronisation, timed on the host (median of `reps`
 * after one untimed run); colptr(B) of every trial is compared with the first one and
 * a trial that differs (or fails) is not chosen.
 */
#ifndef SPKADD_TUNE_H
#define SPKADD_TUNE_H

#include "spkadd.h"
#include "spkadd_batch.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Shape class of an SpKAdd: the device, the value type and the orders of magnitude
 * of m, n, k and of the mean input entries per column; kind tells one SpKAdd from a
 * set of batched requests. */
typedef struct spkadd_tune_key {
  char arch[64];   /* device architecture name (hipDeviceProp_t.gcnArchName) */
  int32_t cus;     /* compute units */
  int32_t dtype;   /* spkadd_dtype */
  int32_t m_log2;  /* ceil(log2(m)), 0 for m <= 1; likewise n and k */
  int32_t n_log2;
  int32_t k_log2;
  int32_t u_log2;  /* ceil(log2(nnz_in / n)) (0 for n == 0 or nnz_in <= n) */
  int32_t kind;    /* 0: one SpKAdd (spkadd_tune); 1: a set of batched requests
                      (spkadd_tune_batch), m, n, k and u then their means */
} spkadd_tune_key;

/* The key of an SpKAdd on the current device.  Errors: INVALID, HIP. */
spkadd_status spkadd_tune_key_for(int32_t m, int32_t n, int32_t k, int64_t nnz_in, spkadd_dtype dtype,
                                  spkadd_tune_key* out);

/* One measured setting. */
typedef struct spkadd_tune_trial {
  spkadd_opts opts;
  double ms;           /* median time of the whole call sequence, < 0 if not timed */
  int32_t status;      /* spkadd_status of the trial */
  int32_t same_colptr; /* 1 if colptr(B) equals the first trial's */
} spkadd_tune_trial;

typedef struct spkadd_tune_report {
  int32_t trials;      /* settings measured */
  int32_t failed;      /* settings that failed or gave another colptr(B) */
  double default_ms;   /* the starting opts */
  double best_ms;      /* the chosen opts */
  spkadd_tune_key key; /* the cache entry written */
} spkadd_tune_report;

/*
 * spkadd_tune -- measure settings on the given inputs (same arguments as spkadd_plan
 * and spkadd_numeric), write the fastest to *best (other fields as in *base) and to
 * the cache under the inputs' key.
 *   base       : starting opts (NULL: defaults); its flags are kept in every trial.
 *   reps       : timed runs per setting (1..100).
 *   trials     : NULL, or a HOST array of max_trials entries filled with the settings
 *                measured, in order.
 * The tuner allocates the outputs (colptr(B), and sum_i nnz(A_i) rows and values) on
 * the device for the duration of the call and synchronises `stream`.
 * Errors: INVALID, OOM, HIP, or the status of the starting setting if it fails.
 */
spkadd_status spkadd_tune(int32_t m, int32_t n, int32_t k, const int32_t* const* colptr, const int32_t* const* rowidx,
                          const void* const* values, spkadd_dtype dtype, const spkadd_opts* base, int32_t reps,
                          spkadd_opts* best, spkadd_tune_report* report, spkadd_tune_trial* trials,
                          int32_t max_trials, hipStream_t stream);

/* The key (kind 1) of a set of batched requests on the current device: nreq requests
 * whose m, n and k add up to sum_m, sum_n, sum_k, with nnz_in input entries in all.
 * Errors: INVALID, HIP. */
spkadd_status spkadd_tune_key_for_batch(int32_t nreq, int64_t sum_m, int64_t sum_n, int64_t sum_k, int64_t nnz_in,
                                        spkadd_dtype dtype, spkadd_tune_key* out);

/*
 * spkadd_tune_batch -- the batched path's counterpart of spkadd_tune: measures
 * settings of the batched runs (spkadd_batch.h) on a sample of requests and keeps the
 * fastest under the sample's key (kind 1).  Searched, one parameter at a time from
 * *base: the requests per run (batch_run_size: 8, 16, 32, 64), the wavefront and
 * workgroup cutoffs (batch_wave_max: 1024, 768, 512; batch_wg_max: 4096, 3072, 2048),
 * the wavefront accumulator (bitmap_ratio 1, 0.5, 2, 4, or hash tables), one fused
 * launch per pass or one per slot (batch_fused_cols 0 / -1) and the workgroup size
 * (batch_wg_threads 256 / 512).  A trial runs every request: runs of batch_run_size
 * requests through two batch objects that alternate (graphs captured in an untimed
 * first pass), then the requests a run reports too large through the one-request
 * path, as the serving loop does; its time is the median of `reps` passes, and
 * nnz(B_r) of every request must equal the first trial's.
 *   reqs, nreq : the sample (as spkadd_batch_run; outputs are written by every trial).
 *   best       : receives *base with the tuned fields (batch_run_size included).
 * Errors: INVALID, OOM, HIP, or the status of the starting setting if it fails.
 */
spkadd_status spkadd_tune_batch(const spkadd_request* reqs, int32_t nreq, spkadd_dtype dtype,
                                const spkadd_opts* base, int32_t reps, spkadd_opts* best,
                                spkadd_tune_report* report, spkadd_tune_trial* trials, int32_t max_trials,
                                hipStream_t stream);

/* Applies the cached setting of *key to *inout (the tuned fields only; flags and test
 * hooks stay).  *found = 1 if there was one, 0 otherwise (then *inout is unchanged).
 * Needs no device.  Errors: INVALID. */
spkadd_status spkadd_tune_lookup(const spkadd_tune_key* key, spkadd_opts* inout, int32_t* found);

/* Stores the tuned fields of *opts under *key (replacing an entry).  Errors: INVALID. */
spkadd_status spkadd_tune_store(const spkadd_tune_key* key, const spkadd_opts* opts, double ms);

/* Entries in the cache. */
int32_t spkadd_tune_size(void);

/* Writes the cache as JSON.  Errors: INVALID (NULL path), STATE (cannot write). */
spkadd_status spkadd_tune_save(const char* path);

/* Reads a JSON file written by spkadd_tune_save and merges its entries into the cache
 * (entries of the file replace those with the same key).  On a malformed file nothing
 * is merged.  Errors: INVALID (NULL path or malformed file), STATE (cannot read). */
spkadd_status spkadd_tune_load(const char* path);

/* Empties the cache. */
void spkadd_tune_clear(void);

#ifdef __cplusplus
}
#endif
#endif /* SPKADD_TUNE_H */
