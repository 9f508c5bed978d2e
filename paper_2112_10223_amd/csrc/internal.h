// Internal interface between the host orchestration (spkadd.cpp) and the HIP
// kernels (plan_kernels.hip, hash_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spkadd.h"

namespace spk {

// Column bins.  A column's bin is chosen from its upper bound
// u_j = sum_i nnz(A_i(:,j)) (the per-column load measure of Section III-A).
//   EMPTY      u_j = 0, nothing to do.
//   W<E>       one wavefront per column, E entries per lane (u_j <= 64 E).
//   G1, G2     one workgroup per column (256 / 512 threads).
//   WIN        the column is cut into row windows (sliding hash, Section III-B);
//              one workgroup per window.
enum Bin : int {
  BIN_EMPTY = 0,
  BIN_W1, BIN_W2, BIN_W3, BIN_W4, BIN_W5, BIN_W6, BIN_W8, BIN_W10, BIN_W12, BIN_W16,
  BIN_G1, BIN_G2,
  BIN_WIN,
  NBINS
};
constexpr int NWAVE_BINS = 10;
__host__ __device__ constexpr int wave_bin_E(int b) {
  return b == BIN_W1 ? 1 : b == BIN_W2 ? 2 : b == BIN_W3 ? 3 : b == BIN_W4 ? 4 : b == BIN_W5 ? 5
       : b == BIN_W6 ? 6 : b == BIN_W8 ? 8 : b == BIN_W10 ? 10 : b == BIN_W12 ? 12 : 16;
}

// Device error bits (plan->d_err).
enum : int {
  ERR_PROBE = 1,      // a hash table ran out of slots (sizing bug)
  ERR_COUNT = 2,      // numeric entry count differs from the symbolic count
  ERR_INPUT = 4,      // validation found a malformed input
  ERR_OVERFLOW = 8,   // a count exceeds int32
};

// Threads of the workgroup bins.
constexpr int G1_THREADS = 256;
constexpr int G2_THREADS = 512;
constexpr int WAVES_PER_BLOCK = 4;   // wave bins (hash kernels): columns per 256-thread block
constexpr int PIPE_WAVES_PER_BLOCK = 4;  // pipelined wave kernels: the wavefronts of a workgroup share
                                         // the CU L1 for neighbouring columns
constexpr int PLAN_THREADS = 256;

struct PlanParams {
  int m, n, k;
  int wave_max;     // largest u_j of the wave bins
  int g1_max;       // largest u_j of bin G1
  int cap_in;       // largest input count of a G2 column or a window
  int force_bin;    // -1 auto
  float win_fill;   // target window input count = cap_in * win_fill
  int unsorted_in;  // input columns may be unsorted (validation checks only the row range)
  int win_min;      // fewest windows of a window column (each then at most the bitmap's rows)
  int win_span;     // widest window left unsplit (the workgroup bitmap's rows; INT32_MAX without bitmaps)
};

// Summary written by the plan kernels; the host reads it from a pinned slot.
struct PlanSummary {
  unsigned long long nnz_in;
  long long total;   // result of the last scan (nnz(B), or the refined window count)
  int err;
  int bin_count[NBINS];
  int n_windows;
  int pad;       // windows still to refine (one refinement level)
  int max_span;  // widest window (rows) of the last level counted
  int pad2;
};

// Arguments of the per-unit symbolic / numeric kernels.
struct KArgs {
  const int* const* cp;   // k device colptr pointers
  const int* const* ri;   // k device rowidx pointers
  const void* const* va;  // k device value pointers (numeric)
  int m, n, k;
  int ktop;               // largest power of two <= k-1 (0 when k == 1)
  int hash_mode;
  int alpha_q;            // table load factor of this phase, in 1/1024
  int* colcnt;            // symbolic: per-column nnz(B(:,j))
  const int* colptr_c;    // numeric: colptr(B)
  int* out_r;             // numeric: rowidx(B)
  void* out_v;            // numeric: values(B)
  // windows
  const int* wcols;       // window column list (column ids)
  const int* win_c;       // window -> index into wcols
  const int* brow;        // boundary rows; window w spans boundaries w + win_c[w] and the next
  const int4* wrec;       // per window: column id, first row, end row, lower boundary index
  const int* bpos;        // boundary positions, k per boundary
  const int* cntin;       // window input entry counts
  int* win_cnt;           // symbolic: per-window unique rows
  const int* win_off;     // numeric: offset of the window inside its output column
  int* err;
  const void* dummy;      // 4 KiB: bytes [0,2048) read as zeros by masked-off loads, [2048,4096) write sink
  int upw;                // wave pipeline: units per wavefront
  // LDS layout (bytes, per wave for the wave kernels, per block for the workgroup kernels)
  int ts_max;             // table slots available
  int off_P, off_adj, off_adjv, off_hist, off_match, off_mark, slice_bytes;
  int bm_nq;              // wave bitmap mode: bitmap rows of 256 words (0 = hash mode)
  int off_bm, off_pre, off_bvals, off_brows;
  // workgroup units: units at most wg_span_max rows wide go to the bitmap kernel (the
  // hash kernel skips them); wg_cap = its staging capacity in output entries
  int wg_span_max, wg_cap;
  int wg_overlay;         // the staging area may overlay the bitmap (ranks read first)
  int wg_group;           // bitmap words per prefix entry (2 or 4)
  int unsorted;           // numeric: 1 = write each column in table order (no sort)
};

}  // namespace spk

// ---- plan kernels (plan_kernels.hip, unsorted_kernels.hip): host launchers ----
#include "plan_launch.h"

namespace spk {

// ---- hash kernels (hash_kernels.hip) ----
// LDS bytes needed by one unit of bin b for a phase (per wave for wave bins).
void lds_layout(int bin, bool numeric, int vbytes, int k, int ts_max, KArgs& a);
// Table slots needed for up to `entries` entries at load factor alpha_q / 1024.
int table_slots(int entries, int alpha_q);
int alpha_to_q(float alpha);
int bin_threads(int bin);
int bin_units_per_block(int bin);
// Launch the symbolic (numeric == false) or numeric kernel of bin b over units
// list[0..nunits) (windows: list == nullptr and units are window ids).
hipError_t launch_hash(int bin, bool numeric, bool f64, const KArgs& a, const int* d_list, int nunits,
                       hipStream_t s);
const char* hash_kernel_name(int bin, bool numeric);
// Pipelined wave-bin kernels (wave_kernels.hip): k <= 64 and numeric load factor 1/2.
bool wave_pipe_ok(int k, int alpha_num_q);
void lds_layout_pipe(int bin, bool numeric, int vbytes, int ts_max, int bm_nq, KArgs& a);
// Workgroup bitmap kernel (bitmap_wg.hip): widest unit it takes (rows), LDS layout,
// launch over a bin's units (G1, G2 or WIN).
int bitmap_wg_span_max();
// one_max: a unit with at most this many entries keeps them all in registers (the
// launch's threads x entries per thread); all_one: every unit of the launch does.
void lds_layout_bitmap_wg(bool numeric, int vbytes, int k, int span_max, int cap, int one_max, bool all_one, int G,
                          KArgs& a);
int bitmap_wg_regs(int bin);
hipError_t launch_bitmap_wg(int bin, bool numeric, bool f64, const KArgs& a, const int* d_list, int nunits,
                            hipStream_t s);
hipError_t launch_wave_pipe(int bin, bool numeric, bool f64, const KArgs& a, const int* d_list, int nunits,
                            hipStream_t s);
int max_lds_bytes();

// Sets the calling thread's spkadd_last_error message and returns st (spkadd.cpp).
spkadd_status report_error(spkadd_status st, const char* msg);

}  // namespace spk
