// Host launchers of the plan kernels (plan_kernels.hip, unsorted_kernels.hip): the
// binning, row-window and scan passes between the plan's host code (spkadd.cpp) and
// the kernels.  Included by internal.h after the shared structures.
#pragma once
#include "internal.h"

namespace spk {

// Device pointers passed by value (kernel arguments) to k_put_ptrs.
struct PtrChunk {
  static constexpr int kMax = 128;
  const void* p[kMax];
  int count;
};

void launch_put_ptrs(const void* const* host_ptrs, int count, const void** d_dst, PlanSummary* d_sum,
                     void* d_dummy, hipStream_t s);
void launch_bounds(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int* d_u,
                   unsigned char* d_bin, int* d_colcnt, int* d_hist, PlanSummary* d_sum, hipStream_t s);
void launch_validate(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, PlanSummary* d_sum,
                     hipStream_t s);
// d_binoff holds 2 NBINS + 1 ints: offsets (NBINS + 1), then the merge map.
void launch_bin_scan(int nblk, bool merge, int* d_hist, int* d_binoff, PlanSummary* d_sum, hipStream_t s);
void launch_bin_scatter(const PlanParams& p, const unsigned char* d_bin, const int* d_hist, const int* d_binoff,
                        int* d_list, hipStream_t s);
void launch_win_scan(const PlanParams& p, const int* d_list, const int* d_binoff, const int* d_u, int* d_wfirst,
                     PlanSummary* d_sum, hipStream_t s);
// First windows of the window columns: row quantiles of each column's longest input
// (sorted inputs), else equal row ranges.
void launch_win_fill(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, const int* d_wcols,
                     const int* d_u, int n_wcols, const int* d_wfirst, int* d_win_c, int* d_brow, int* d_bcol,
                     int* d_wlin, hipStream_t s);
// Every boundary's position in every input: for the columns of the ordered pass
// (win_search_linear) one wavefront per input writing d_bpos; for the others one pass
// over their entries in the chunks of launch_uwin_chunks / launch_uwin_chfill into
// d_bpos_t (input-major, the size of d_bpos), then transposed into d_bpos.
void launch_win_search(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, const int* d_wcols,
                       const int* d_wfirst, const int* d_wlin, int n_wcols, const int* d_brow, const int* d_bcol,
                       int n_bounds, int n_chunks, const int* d_chfirst, const int* d_chcol, int* d_bpos_t,
                       int* d_bpos, hipStream_t s);
void launch_win_records(int n_windows, const int* d_wcols, const int* d_win_c, const int* d_brow, int4* d_wrec,
                        hipStream_t s);
// Whether window column c may keep equal row splits found by one ordered pass per
// input with the window of a row computed arithmetically (k_win_search_lin): when each
// input holds 1024..8192 rows of the column on average (long sorted runs that one
// wavefront walks at streaming speed), and k_win_fill finds the equal splits about
// balanced; other columns take row quantiles and the chunked pass (k_win_locate).
__host__ __device__ inline bool win_search_linear(long long u, int k) { return u >= 1024LL * k && u <= 8192LL * k; }

// Work units of the passes over the window columns' entries (the boundary positions
// of sorted inputs, the window histogram of unsorted ones): chunks of a column's
// concatenated input segments, or one chunk per column when it has more than
// WIN_LDS_K inputs (more than the on-chip segment table).
constexpr int WIN_CHUNK = 4096;       // unsorted inputs' passes
constexpr int WIN_LOC_CHUNK = 16384;  // boundary positions of sorted inputs
constexpr int WIN_LDS_K = 1024;
// Unsorted input (unsorted_kernels.hip): window counts by histogram, the bucket
// partition of the final windows, and the numeric pass's value gather.
// d_wlin: no chunk for the columns of the ordered pass (d_wlin[c] set by launch_win_fill),
// or nullptr
void launch_uwin_chunks(const PlanParams& p, int n_wcols, const int* d_wcols, const int* d_u, int chunk,
                        const int* d_wlin, int* d_nch, hipStream_t s);
void launch_uwin_chfill(int n_wcols, const int* d_chfirst, int* d_chcol, hipStream_t s);
void launch_uwin_hist(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int n_chunks,
                      const int* d_wcols, const int* d_wfirst, const int* d_brow, const int* d_chfirst,
                      const int* d_chcol, int* d_cnt, hipStream_t s);
void launch_uwin_scatter(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int n_chunks,
                         const int* d_wcols, const int* d_wfirst, const int* d_brow, const int* d_chfirst,
                         const int* d_chcol, int* d_gcur, int* d_brows, long long* d_bsrc, hipStream_t s);
void launch_uwin_bpos(int n_windows, const int* d_win_c, const int* d_wfirst, const int* d_boff, int* d_bpos,
                      hipStream_t s);
void launch_uwin_gather(long long total, const long long* d_bsrc, const void* const* d_va, void* d_bvals, bool f64,
                        hipStream_t s);
// d_bpos NULL: the counts are already in d_cntin (unsorted input)
void launch_win_count(const PlanParams& p, int n_windows, const int* d_win_c, const int* d_brow, const int* d_bpos,
                      int* d_cntin, int* d_q, PlanSummary* d_sum, hipStream_t s);
// One refinement level (d_bpos_old: the boundary positions of sorted inputs, which let
// a window be cut at row quantiles; nullptr: equal row ranges).
void launch_win_refine_fill(const PlanParams& p, int n_windows, int n_wcols, const int* d_win_c,
                            const int* d_wfirst_old, const int* d_q, const int* d_newfirst, const int* d_brow_old,
                            const int* const* d_ri, const int* d_bpos_old, int* d_win_c_new, int* d_brow_new,
                            int* d_bcol_new, int* d_bpar, int* d_bpiece, int* d_wfirst_new, hipStream_t s);
void launch_win_refine_search(const PlanParams& p, const int* const* d_ri, int n_bounds_new, const int* d_bcol_new,
                              const int* d_brow_new, const int* d_bpar, const int* d_bpiece, const int* d_q,
                              const int* d_bpos_old, int* d_bpos_new, hipStream_t s);
void launch_win_colsum(int n_wcols, const int* d_wcols, const int* d_wfirst, const int* d_win_cnt, int* d_colcnt,
                       int* d_win_off, hipStream_t s);

// Exclusive scan of len int32 counts into out[0..len] (out[len] = total).  The total
// is also stored as int64 in *d_total; totals above INT32_MAX set ERR_OVERFLOW in
// *d_err and leave out[] unspecified.  d_tmp needs scan_tmp_bytes(len).
size_t scan_tmp_bytes(int64_t len);
void launch_scan(const int* d_in, int64_t len, int* d_out, long long* d_total, int* d_err, void* d_tmp,
                 hipStream_t s);

}  // namespace spk
