/*
 * spkadd_baselines.h -- the paper's comparison algorithm for SpKAdd, on the GPU, for
 * measuring the hash method against (not the product path; spkadd.h is).
 *
 * spkadd_heap_add -- B = A_1 + ... + A_k by the k-way heap merge of Algorithm 3
 * (HeapAdd, Section II-C): per column, a min-heap holding the current entry of every
 * input; the smallest row is popped, added to B(:, j) (a new output entry when its row
 * differs from the last one written) and replaced by the next entry of its input.
 * One GPU thread merges one column, its heap in LDS; a symbolic pass counts the
 * distinct rows, a scan gives colptr(B), a numeric pass writes B.
 *
 * (The other baseline of the paper's comparison, the 2-way tree of Section II-B, is
 * built from spkadd.h itself: lg k rounds of k = 2 sums; paper_2112_10223_amd/
 * baselines.py.)
 *
 * Arguments (memory rules of spkadd.h: HOST arrays of k DEVICE pointers, DEVICE
 * outputs; the caller owns everything):
 *   m, n, k    : shape and number of inputs, 1 <= k <= SPKADD_HEAP_MAX_K.
 *   colptr     : k pointers to int32[n+1]; rowidx: k pointers to int32 rows, strictly
 *                ascending within each column (the merge needs sorted inputs).
 *   values     : k pointers to float or double (dtype).
 *   colptr_c   : DEVICE int32[n+1], written with colptr(B).
 *   rowidx_c, values_c : DEVICE arrays of cap_c entries; written only when
 *                nnz(B) <= cap_c (sum of the inputs' nnz is always enough).
 *   nnz_c      : HOST, receives nnz(B).  The call waits for the count on `stream`
 *                and then enqueues the numeric pass asynchronously.
 * Errors: INVALID (NULL arrays, k out of range, bad shape), OVERFLOW (nnz(B) above
 * INT32_MAX), OOM, HIP.  nnz(B) > cap_c is not an error: *nnz_c tells the caller.
 */
#ifndef SPKADD_BASELINES_H
#define SPKADD_BASELINES_H

#include "spkadd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SPKADD_HEAP_MAX_K 128

spkadd_status spkadd_heap_add(int32_t m, int32_t n, int32_t k, const int32_t* const* colptr,
                              const int32_t* const* rowidx, const void* const* values, spkadd_dtype dtype,
                              int32_t* colptr_c, int32_t* rowidx_c, void* values_c, int64_t cap_c, int64_t* nnz_c,
                              hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif
