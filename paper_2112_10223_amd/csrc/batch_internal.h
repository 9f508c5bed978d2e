// Internal interface of the batched launch (batch.cpp <-> batch_kernels.hip).
#pragma once
#include "internal.h"

namespace spk {

// Request descriptor as the device sees it (written by the host into a pinned
// table, copied to the device at the start of a run).
struct BatchReq {
  const int* const* cp;   // device table of k colptr pointers
  const int* const* ri;   // device table of k rowidx pointers
  const void* const* va;  // device table of k value pointers
  int* colptr_c;
  int* out_r;
  void* out_v;
  long long cap;          // output capacity in entries
  int m, n, k;
  int col_base;           // global index of the request's column 0
  int nq;                 // bitmap rows of 256 words (ceil(m / 8192)), 0 = no bitmap
  int pad[3];
};

struct BatchHdr {
  int nreq;
  int total_cols;
  int pad[2];
};

// Column slots: empty, too large for a wavefront, then (wave bin, accumulator).
constexpr int BSLOT_EMPTY = 0;
constexpr int BSLOT_LARGE = 1;
constexpr int BSLOT_WAVE = 2;  // + 2 * (wave bin index) + (1 for the bitmap)
// Workgroup-sized columns (wave_max < u_j <= wg_max <= BATCH_WG_U, by default 1024
// and 4096) of requests with at most BATCH_WG_SPAN rows: one workgroup bitmap each
// (larger columns are left to the one-request path).
constexpr int BSLOT_WG = BSLOT_WAVE + 2 * NWAVE_BINS;
constexpr int BSLOTS = BSLOT_WG + 1;
constexpr int BATCH_WG_U = 4096;
constexpr int BATCH_WG_SPAN = 1 << 17;
constexpr int BATCH_WG_THREADS = 256;  // default threads per workgroup of the workgroup slot (256 or 512)
constexpr int BATCH_SCAN_THREADS = 1024;  // one workgroup per request scans its column counts
constexpr int BATCH_MAX_BOUNDS_BLOCKS = 1024;
constexpr int BATCH_CHUNK = 16;  // list entries per wavefront task

// Per-request outcome bits (values of SPKADD_REQ_*).
enum : int { REQ_TOO_LARGE = 1, REQ_CAPACITY = 2 };

struct BatchArgs {
  const BatchHdr* hdr;
  const BatchReq* reqs;
  int* req_of;          // per global column
  unsigned char* slot;  // per global column
  int* colcnt;          // per global column: nnz(B(:,j))
  int* hist;            // per bounds block x BSLOTS
  int* slotoff;         // BSLOTS + 1 offsets, then BSLOTS counts
  int* list;            // global column ids by slot
  long long* nnz;       // per request
  int* status;          // per request
  int* err;
  const void* dummy;    // 4 KiB: [0, 2048) zeros, [2048, 4096) write sink
  int max_reqs;
  int nblk;             // bounds / scatter blocks
  int chunk;            // columns per bounds block (multiple of 256)
  int accum_mode;
  float bitmap_ratio;
  int wave_max;         // largest u_j of a wavefront slot
  int wg_max;           // largest u_j of the workgroup slot (larger: the request is too large)
};

void launch_batch_plan(const BatchArgs& b, hipStream_t s);
void launch_batch_scan(const BatchArgs& b, hipStream_t s);
void launch_batch_wave(int wi, bool numeric, bool f64, bool bm, const BatchArgs& b, const KArgs& a, unsigned blocks,
                       size_t lds, hipStream_t s);
// Every wave slot of one pass in one launch; `a` holds the common fields and the
// LDS slice (the largest of the slots).
void launch_batch_fused(bool numeric, bool f64, const BatchArgs& b, const KArgs& a, unsigned blocks, size_t lds,
                        hipStream_t s);
// The workgroup-sized columns of one pass; `a` holds the common fields and the LDS
// layout (lds_layout_bitmap_wg for BATCH_WG_SPAN rows, BATCH_WG_U entries, k = 64).
void launch_batch_wg(bool numeric, bool f64, int threads, const BatchArgs& b, const KArgs& a, unsigned blocks,
                     hipStream_t s);
// Blocks of the fused kernel resident per CU with `lds` bytes of LDS per block (0 if
// the query fails).
int batch_fused_blocks_per_cu(bool numeric, bool f64, size_t lds);
// LDS layout of a wave slice (same as the plain launch).
void lds_layout_pipe(int bin, bool numeric, int vbytes, int ts_max, int bm_nq, KArgs& a);

}  // namespace spk
