// Host side of the batched SpKAdd (include/spkadd_batch.h): request validation, the
// request table (pinned host buffer -> device, one copy per run), the fixed launch
// sequence, its capture as a hipGraph per launch shape, and the per-request results.
#include "spkadd_batch.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "batch_internal.h"

using namespace spk;

namespace {

spkadd_status fail(spkadd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return report_error(st, buf);
}

#define BHIP(expr)                                                                                         \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess) {                                                                                \
      (void)hipGetLastError();                                                                             \
      return fail(SPKADD_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    }                                                                                                      \
  } while (0)

// What a launch sequence depends on besides device data: the largest bitmap of the
// requests that may use one (rounded up to a power of two), and which (wave bin,
// accumulator) launches can occur.  A sequence captured for a key also serves every
// key it covers: a launch with no columns of its kind exits at once.
struct ShapeKey {
  int fused;  // 1: one launch per pass for every wave slot
  int nq_max;
  unsigned bm_mask, hash_mask;
  bool operator<(const ShapeKey& o) const {
    if (fused != o.fused) return fused < o.fused;
    if (nq_max != o.nq_max) return nq_max < o.nq_max;
    if (bm_mask != o.bm_mask) return bm_mask < o.bm_mask;
    return hash_mask < o.hash_mask;
  }
  bool covers(const ShapeKey& o) const {
    return fused == o.fused && nq_max >= o.nq_max && (o.bm_mask & ~bm_mask) == 0 && (o.hash_mask & ~hash_mask) == 0;
  }
  int launches() const { return __builtin_popcount(bm_mask) + __builtin_popcount(hash_mask); }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct spkadd_batch_s {
  int device = 0;
  spkadd_dtype dtype = SPKADD_F32;
  spkadd_opts opts{};
  int max_reqs = 0;
  long long max_cols = 0, max_inputs = 0;
  int n_cu = 256;
  // device workspace (one allocation)
  char* d_ws = nullptr;
  char* d_blob = nullptr;  // BatchHdr, BatchReq[max_reqs], pointer tables
  // pinned host
  char* h_blob = nullptr;
  size_t blob_bytes = 0;
  // per-request results: nnz, status and the error flags, one device region and its
  // pinned mirror with the same layout, copied back in one transfer
  char* d_res = nullptr;
  char* h_res = nullptr;
  size_t res_bytes = 0;
  long long* h_nnz = nullptr;
  int* h_status = nullptr;
  int* h_err = nullptr;
  hipEvent_t ev_upload = nullptr, ev_done = nullptr;
  bool upload_pending = false;
  hipStream_t cap_stream = nullptr;
  std::map<ShapeKey, hipGraphExec_t> graphs;
  int graph_reuses = 0;  // runs served by a graph captured for a covering key
  long long fused_cols = INT32_MAX;  // runs with at most this many columns use the fused launches (< 0: never)
  int fused_runs = 0;
  BatchArgs args{};
  int last_nreq = -1;
  int graph_replays = 0;
  int kernels_per_run = 0;
  int wg_threads = BATCH_WG_THREADS;
};

namespace {

size_t blob_size(int max_reqs, long long max_inputs) {
  return align_up(sizeof(BatchHdr), 64) + align_up((size_t)max_reqs * sizeof(BatchReq), 64) +
         (size_t)3 * (size_t)max_inputs * sizeof(void*);
}

// Bitmap rows of a request's bitmap, 0 when its rows do not fit one (m > 131072).
int request_nq(int m) { return (m > 0 && m <= 131072) ? (m + 8191) / 8192 : 0; }

bool bitmap_for(const spkadd_opts& o, int nq, int E) {
  if (o.accum_mode == SPKADD_ACCUM_HASH || nq <= 0) return false;
  if (o.accum_mode == SPKADD_ACCUM_BITMAP) return true;
  const float ratio = o.bitmap_ratio > 0 ? o.bitmap_ratio : 1.0f;
  return (float)nq <= ratio * (float)E;
}

// The launch arguments of one (wave bin, accumulator) slot of a pass: common fields
// and the LDS layout of its slice.
KArgs slot_args(const spkadd_batch_s* b, const ShapeKey& key, int wi, bool bm, bool numeric) {
  const int vb = b->dtype == SPKADD_F64 ? 8 : 4;
  const int bin = BIN_W1 + wi;
  KArgs a{};
  a.err = b->args.err;
  a.dummy = b->args.dummy;
  a.alpha_q = 512;
  a.hash_mode = 0;
  a.upw = 1;
  const int ts = table_slots(64 * wave_bin_E(bin), 512);
  // the largest bitmap a column of this bin can use: with the automatic choice
  // only bitmaps of at most bitmap_ratio * E rows of 8192 bits
  int nq_bin = key.nq_max;
  if (bm && b->args.accum_mode == SPKADD_ACCUM_AUTO)
    while (nq_bin > 1 && !((float)nq_bin <= b->args.bitmap_ratio * (float)wave_bin_E(bin))) --nq_bin;
  lds_layout_pipe(bin, numeric, vb, ts, bm ? nq_bin : 0, a);
  if (bm) {
    // each request lays out its own slice for its bitmap size; a smaller bitmap
    // can need more room (its staged rows and values may not fit over it), so
    // the launch slice is the largest over every size up to the bin's maximum
    for (int nq = 1; nq < nq_bin; ++nq) {
      KArgs t{};
      lds_layout_pipe(bin, numeric, vb, ts, nq, t);
      if (t.slice_bytes > a.slice_bytes) a.slice_bytes = t.slice_bytes;
    }
  }
  return a;
}

unsigned grid_for(const spkadd_batch_s* b, int slice_bytes, int* block_lds) {
  *block_lds = slice_bytes * PIPE_WAVES_PER_BLOCK;
  int bpc = max_lds_bytes() / *block_lds;
  if (bpc > 16 / PIPE_WAVES_PER_BLOCK) bpc = 16 / PIPE_WAVES_PER_BLOCK;
  if (bpc < 1) bpc = 1;
  return (unsigned)(b->n_cu * bpc);
}

// The workgroup-sized columns of a pass (every run: whether a run has any is known on
// the device only).
int enqueue_wg(spkadd_batch_s* b, bool numeric, hipStream_t s) {
  const bool f64 = b->dtype == SPKADD_F64;
  KArgs a{};
  a.err = b->args.err;
  a.dummy = b->args.dummy;
  a.alpha_q = 512;
  // every workgroup-slot column has at most wg_max (<= BATCH_WG_U) entries, all in
  // registers: the staging area holds wg_max of them
  lds_layout_bitmap_wg(numeric, f64 ? 8 : 4, 64, BATCH_WG_SPAN, b->args.wg_max, BATCH_WG_U, true, 2, a);
  // resident workgroups per CU: LDS-bound, at most 32 waves
  const int max_blocks = 32 / (b->wg_threads / 64);
  int bpc = max_lds_bytes() / a.slice_bytes;
  bpc = bpc < 1 ? 1 : bpc > max_blocks ? max_blocks : bpc;
  launch_batch_wg(numeric, f64, b->wg_threads, b->args, a, (unsigned)(b->n_cu * bpc), s);
  return 1;
}

// The whole run after the request-table upload.  Returns the kernels enqueued.
int enqueue_run(spkadd_batch_s* b, const ShapeKey& key, hipStream_t s) {
  int kernels = 0;
  const bool f64 = b->dtype == SPKADD_F64;
  launch_batch_plan(b->args, s);
  kernels += 4;
  for (int numeric = 0; numeric < 2; ++numeric) {
    if (numeric) {
      launch_batch_scan(b->args, s);
      ++kernels;
    }
    kernels += enqueue_wg(b, numeric != 0, s);
    if (key.fused) {
      // one launch: the slice is the largest of the slots that can occur
      KArgs a{};
      bool any = false;
      for (int wi = 0; wi < NWAVE_BINS; ++wi)
        for (int bm = 0; bm < 2; ++bm) {
          if (!((bm ? key.bm_mask : key.hash_mask) >> wi & 1u)) continue;
          const KArgs t = slot_args(b, key, wi, bm != 0, numeric != 0);
          if (!any || t.slice_bytes > a.slice_bytes) a = t;
          any = true;
        }
      if (!any) continue;
      int block_lds = 0;
      unsigned blocks = grid_for(b, a.slice_bytes, &block_lds);
      // persistent: no more blocks than can be resident at once (registers can
      // limit this kernel more than LDS)
      const int occ = batch_fused_blocks_per_cu(numeric != 0, f64, (size_t)block_lds);
      if (occ > 0 && blocks > (unsigned)(b->n_cu * occ)) blocks = (unsigned)(b->n_cu * occ);
      launch_batch_fused(numeric != 0, f64, b->args, a, blocks, (size_t)block_lds, s);
      ++kernels;
      continue;
    }
    for (int wi = 0; wi < NWAVE_BINS; ++wi) {
      for (int bm = 0; bm < 2; ++bm) {
        if (!((bm ? key.bm_mask : key.hash_mask) >> wi & 1u)) continue;
        const KArgs a = slot_args(b, key, wi, bm != 0, numeric != 0);
        int block_lds = 0;
        const unsigned blocks = grid_for(b, a.slice_bytes, &block_lds);
        launch_batch_wave(wi, numeric != 0, f64, bm != 0, b->args, a, blocks, (size_t)block_lds, s);
        ++kernels;
      }
    }
  }
  return kernels;
}

void destroy(spkadd_batch_s* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->ev_upload) (void)hipEventDestroy(b->ev_upload);
  if (b->ev_done) (void)hipEventDestroy(b->ev_done);
  if (b->d_ws) (void)hipFree(b->d_ws);
  if (b->h_blob) (void)hipHostFree(b->h_blob);
  delete b;
}

}  // namespace

extern "C" {

spkadd_status spkadd_batch_create(spkadd_batch_t* out, spkadd_dtype dtype, int32_t max_requests,
                                  int64_t max_columns, int64_t max_inputs, const spkadd_opts* opts) {
  if (!out) return fail(SPKADD_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (dtype != SPKADD_F32 && dtype != SPKADD_F64) return fail(SPKADD_ERR_INVALID, "bad dtype %d", (int)dtype);
  if (max_requests < 1 || max_columns < 1 || max_inputs < 1)
    return fail(SPKADD_ERR_INVALID, "max_requests, max_columns and max_inputs must be >= 1");
  if (max_columns > (1LL << 30) || max_inputs > (1LL << 26) || max_requests > (1 << 24))
    return fail(SPKADD_ERR_INVALID, "batch limits too large");
  spkadd_opts o;
  spkadd_opts_default(&o);
  if (opts) o = *opts;
  if (o.accum_mode < 0 || o.accum_mode > 2) return fail(SPKADD_ERR_INVALID, "bad accum_mode %d", o.accum_mode);
  if (!(o.bitmap_ratio >= 0.f && o.bitmap_ratio <= 64.f)) return fail(SPKADD_ERR_INVALID, "bad bitmap_ratio");
  if (o.flags & SPKADD_FLAG_ORDERED)
    return fail(SPKADD_ERR_UNSUPPORTED, "batched runs do not take SPKADD_FLAG_ORDERED (use spkadd_plan)");
  const int wave_max = o.batch_wave_max ? o.batch_wave_max : 1024;
  const int wg_max = o.batch_wg_max ? o.batch_wg_max : BATCH_WG_U;
  if (wave_max < 64 || wave_max > 1024) return fail(SPKADD_ERR_INVALID, "batch_wave_max must be 0 or 64..1024");
  if (wg_max < wave_max || wg_max > BATCH_WG_U)
    return fail(SPKADD_ERR_INVALID, "batch_wg_max must be 0 or batch_wave_max..%d", BATCH_WG_U);
  if (o.batch_wg_threads != 0 && o.batch_wg_threads != 256 && o.batch_wg_threads != 512)
    return fail(SPKADD_ERR_INVALID, "batch_wg_threads must be 0, 256 or 512");
  if (o.batch_run_size < 0) return fail(SPKADD_ERR_INVALID, "batch_run_size must be >= 0");

  auto* b = new (std::nothrow) spkadd_batch_s();
  if (!b) return fail(SPKADD_ERR_OOM, "host allocation failed");
  b->dtype = dtype;
  b->opts = o;
  b->max_reqs = max_requests;
  b->max_cols = max_columns;
  b->max_inputs = max_inputs;
  b->fused_cols = o.batch_fused_cols == 0 ? (long long)INT32_MAX : o.batch_fused_cols < 0 ? -1 : o.batch_fused_cols;
  auto bail = [&](spkadd_status st, const char* what, hipError_t e) {
    (void)hipGetLastError();
    destroy(b);
    return fail(st, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&b->device))) return bail(SPKADD_ERR_HIP, "hipGetDevice", e);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
    b->n_cu = cus;
  // bounds blocks: at most 1024, each a multiple of 256 columns
  const long long steps = (max_columns + 255) / 256;
  const long long nblk0 = steps < BATCH_MAX_BOUNDS_BLOCKS ? steps : BATCH_MAX_BOUNDS_BLOCKS;
  const int chunk = (int)(256 * ((steps + nblk0 - 1) / nblk0));
  const int nblk = (int)((max_columns + chunk - 1) / chunk);
  b->blob_bytes = blob_size(max_requests, max_inputs);
  const size_t cols = (size_t)max_columns;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o2 = off;
    off += align_up(bytes ? bytes : 1, 256);
    return o2;
  };
  const size_t o_blob = carve(b->blob_bytes), o_reqof = carve(cols * 4), o_slot = carve(cols),
               o_cnt = carve(cols * 4), o_hist = carve((size_t)nblk * BSLOTS * 4),
               o_slotoff = carve((2 * BSLOTS + 1) * 4), o_list = carve(cols * 4),
               o_nnz = carve((size_t)max_requests * 8), o_status = carve((size_t)max_requests * 4), o_err = carve(4),
               o_dummy = carve(4096);
  if ((e = hipMalloc((void**)&b->d_ws, off))) return bail(SPKADD_ERR_OOM, "device workspace", e);
  b->res_bytes = o_err + 4 - o_nnz;
  const size_t h_bytes = align_up(b->blob_bytes, 256) + b->res_bytes;
  if ((e = hipHostMalloc((void**)&b->h_blob, align_up(h_bytes, 4096), hipHostMallocPortable)))
    return bail(SPKADD_ERR_OOM, "pinned host buffer", e);
  b->d_res = b->d_ws + o_nnz;
  b->h_res = b->h_blob + align_up(b->blob_bytes, 256);
  b->h_nnz = (long long*)b->h_res;
  b->h_status = (int*)(b->h_res + (o_status - o_nnz));
  b->h_err = (int*)(b->h_res + (o_err - o_nnz));
  if ((e = hipEventCreateWithFlags(&b->ev_upload, hipEventDisableTiming))) return bail(SPKADD_ERR_HIP, "event", e);
  if ((e = hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming))) return bail(SPKADD_ERR_HIP, "event", e);
  if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking))) return bail(SPKADD_ERR_HIP, "stream", e);
  b->d_blob = b->d_ws + o_blob;
  BatchArgs& a = b->args;
  a.hdr = (const BatchHdr*)b->d_blob;
  a.reqs = (const BatchReq*)(b->d_blob + align_up(sizeof(BatchHdr), 64));
  a.req_of = (int*)(b->d_ws + o_reqof);
  a.slot = (unsigned char*)(b->d_ws + o_slot);
  a.colcnt = (int*)(b->d_ws + o_cnt);
  a.hist = (int*)(b->d_ws + o_hist);
  a.slotoff = (int*)(b->d_ws + o_slotoff);
  a.list = (int*)(b->d_ws + o_list);
  a.nnz = (long long*)(b->d_ws + o_nnz);
  a.status = (int*)(b->d_ws + o_status);
  a.err = (int*)(b->d_ws + o_err);
  a.dummy = b->d_ws + o_dummy;
  a.max_reqs = max_requests;
  a.nblk = nblk;
  a.chunk = chunk;
  a.accum_mode = o.accum_mode;
  a.bitmap_ratio = o.bitmap_ratio > 0 ? o.bitmap_ratio : 1.0f;
  a.wave_max = wave_max;
  a.wg_max = wg_max;
  b->wg_threads = o.batch_wg_threads ? o.batch_wg_threads : BATCH_WG_THREADS;
  *out = b;
  return SPKADD_OK;
}

spkadd_status spkadd_batch_run(spkadd_batch_t b, const spkadd_request* reqs, int32_t nreq, int32_t use_graph,
                               hipStream_t stream) {
  (void)hipGetLastError();  // a stale status of the caller's earlier HIP calls
  if (!b) return fail(SPKADD_ERR_INVALID, "batch is NULL");
  if (nreq < 1 || nreq > b->max_reqs) return fail(SPKADD_ERR_INVALID, "nreq = %d (limit %d)", nreq, b->max_reqs);
  if (!reqs) return fail(SPKADD_ERR_INVALID, "reqs is NULL");
  long long cols = 0, inputs = 0;
  for (int r = 0; r < nreq; ++r) {
    const spkadd_request& q = reqs[r];
    if (q.k < 1 || q.k > 64) return fail(SPKADD_ERR_INVALID, "request %d: k = %d (1..64)", r, q.k);
    if (q.m < 0 || q.n < 0 || q.m == INT32_MAX || q.n == INT32_MAX)
      return fail(SPKADD_ERR_INVALID, "request %d: bad shape", r);
    if (!q.colptr || !q.rowidx || !q.values || !q.colptr_c || q.cap_c < 0)
      return fail(SPKADD_ERR_INVALID, "request %d: NULL array or negative capacity", r);
    if (q.cap_c > 0 && (!q.rowidx_c || !q.values_c))
      return fail(SPKADD_ERR_INVALID, "request %d: NULL output arrays", r);
    for (int i = 0; i < q.k; ++i)
      if (!q.colptr[i] || !q.rowidx[i] || !q.values[i])
        return fail(SPKADD_ERR_INVALID, "request %d: input %d has a NULL array", r, i);
    cols += q.n;
    inputs += q.k;
  }
  if (cols > b->max_cols || cols > INT32_MAX) return fail(SPKADD_ERR_INVALID, "%lld columns (limit %lld)", cols, b->max_cols);
  if (inputs > b->max_inputs) return fail(SPKADD_ERR_INVALID, "%lld inputs (limit %lld)", inputs, b->max_inputs);

  // the previous run's table upload must have left the pinned buffer
  if (b->upload_pending) BHIP(hipEventSynchronize(b->ev_upload));
  ShapeKey key{0, 0, 0u, 0u};
  key.fused = b->fused_cols >= 0 && cols <= b->fused_cols ? 1 : 0;
  char* hb = b->h_blob;
  auto* hdr = (BatchHdr*)hb;
  auto* hq = (BatchReq*)(hb + align_up(sizeof(BatchHdr), 64));
  // the pointer tables follow the descriptors in use, so one copy moves both
  const size_t ptr_off = align_up(sizeof(BatchHdr), 64) + align_up((size_t)nreq * sizeof(BatchReq), 64);
  auto* hp = (const void**)(hb + ptr_off);
  auto* dp = (const void**)(b->d_blob + ptr_off);
  hdr->nreq = nreq;
  hdr->total_cols = (int)cols;
  long long pcur = 0;
  int col_base = 0;
  for (int r = 0; r < nreq; ++r) {
    const spkadd_request& q = reqs[r];
    BatchReq d{};
    d.cp = (const int* const*)(dp + pcur);
    d.ri = (const int* const*)(dp + pcur + q.k);
    d.va = (const void* const*)(dp + pcur + 2 * q.k);
    for (int i = 0; i < q.k; ++i) {
      hp[pcur + i] = q.colptr[i];
      hp[pcur + q.k + i] = q.rowidx[i];
      hp[pcur + 2 * q.k + i] = q.values[i];
    }
    pcur += 3 * q.k;
    d.colptr_c = q.colptr_c;
    d.out_r = q.rowidx_c;
    d.out_v = q.values_c;
    d.cap = q.cap_c;
    d.m = q.m;
    d.n = q.n;
    d.k = q.k;
    d.col_base = col_base;
    col_base += q.n;
    d.nq = request_nq(q.m);
    for (int wi = 0; wi < NWAVE_BINS; ++wi) {
      if (bitmap_for(b->opts, d.nq, wave_bin_E(BIN_W1 + wi))) {
        key.bm_mask |= 1u << wi;
        if (d.nq > key.nq_max) key.nq_max = d.nq;
      } else {
        key.hash_mask |= 1u << wi;
      }
    }
    hq[r] = d;
  }
  if (key.nq_max > 0) {
    int p2 = 1;
    while (p2 < key.nq_max) p2 <<= 1;
    key.nq_max = p2;
  }
  // one copy: header, the descriptors in use and their pointer tables
  BHIP(hipMemcpyAsync(b->d_blob, hb, ptr_off + (size_t)pcur * sizeof(void*), hipMemcpyHostToDevice, stream));
  BHIP(hipEventRecord(b->ev_upload, stream));
  b->upload_pending = true;

  if (use_graph) {
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      // the cheapest captured sequence that covers this run
      for (auto jt = b->graphs.begin(); jt != b->graphs.end(); ++jt)
        if (jt->first.covers(key) && (it == b->graphs.end() || jt->first.launches() < it->first.launches())) it = jt;
      if (it != b->graphs.end()) ++b->graph_reuses;
    }
    if (it == b->graphs.end()) {
      hipGraph_t g = nullptr;
      hipGraphExec_t x = nullptr;
      BHIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      const int kernels = enqueue_run(b, key, b->cap_stream);
      hipError_t le = hipGetLastError();
      // the results copy is part of the graph (fixed addresses and size)
      if (le == hipSuccess)
        le = hipMemcpyAsync(b->h_res, b->d_res, b->res_bytes, hipMemcpyDeviceToHost, b->cap_stream);
      hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return fail(SPKADD_ERR_HIP, "graph capture: %s", hipGetErrorString(le != hipSuccess ? le : ce));
      }
      ce = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ce != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPKADD_ERR_HIP, "graph instantiate: %s", hipGetErrorString(ce));
      }
      it = b->graphs.emplace(key, x).first;
      b->kernels_per_run = kernels;
    }
    BHIP(hipGraphLaunch(it->second, stream));
    ++b->graph_replays;
  } else {
    b->kernels_per_run = enqueue_run(b, key, stream);
    BHIP(hipGetLastError());
    BHIP(hipMemcpyAsync(b->h_res, b->d_res, b->res_bytes, hipMemcpyDeviceToHost, stream));
  }
  BHIP(hipEventRecord(b->ev_done, stream));
  b->last_nreq = nreq;
  b->fused_runs += key.fused;
  return SPKADD_OK;
}

spkadd_status spkadd_batch_results(spkadd_batch_t b, int64_t* nnz, int32_t* status) {
  if (!b) return fail(SPKADD_ERR_INVALID, "batch is NULL");
  if (b->last_nreq < 0) return fail(SPKADD_ERR_STATE, "no run yet");
  BHIP(hipEventSynchronize(b->ev_done));
  if (*b->h_err & (ERR_PROBE | ERR_COUNT))
    return fail(SPKADD_ERR_HIP, "internal error: device flags 0x%x", *b->h_err);
  for (int r = 0; r < b->last_nreq; ++r) {
    if (nnz) nnz[r] = b->h_nnz[r];
    if (status) status[r] = b->h_status[r] & REQ_TOO_LARGE ? SPKADD_REQ_TOO_LARGE
                            : b->h_status[r] & REQ_CAPACITY ? SPKADD_REQ_CAPACITY
                                                            : SPKADD_REQ_OK;
  }
  return SPKADD_OK;
}

int32_t spkadd_batch_ready(spkadd_batch_t b) {
  if (!b || b->last_nreq < 0) return 1;
  const hipError_t e = hipEventQuery(b->ev_done);
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();
    return 0;
  }
  return 1;  // done, or failed (spkadd_batch_results reports it)
}

spkadd_status spkadd_batch_get_info(spkadd_batch_t b, spkadd_batch_info* out) {
  if (!b || !out) return fail(SPKADD_ERR_INVALID, "NULL argument");
  out->graphs_captured = (int32_t)b->graphs.size();
  out->graph_replays = b->graph_replays;
  out->kernels_per_run = b->kernels_per_run;
  out->graph_reuses = b->graph_reuses;
  out->fused_runs = b->fused_runs;
  return SPKADD_OK;
}

spkadd_status spkadd_batch_destroy(spkadd_batch_t b) {
  if (!b) return SPKADD_OK;
  if (b->last_nreq >= 0) (void)hipEventSynchronize(b->ev_done);
  destroy(b);
  return SPKADD_OK;
}

}  // extern "C"
