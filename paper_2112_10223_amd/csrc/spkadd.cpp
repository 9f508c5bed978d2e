// Host side of the SpKAdd C ABI: argument checks, the plan object, the workspace
// cache, and the order of the device passes (plan -> symbolic -> numeric).
#include "spkadd.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "ordered.h"
#include "region.h"
#include "wave_fused.h"

using namespace spk;

namespace {

thread_local std::string g_last_error;

spkadd_status set_error(spkadd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

}  // namespace

namespace spk {
// The thread's last-error message, shared with the batch API (batch.cpp).
spkadd_status report_error(spkadd_status st, const char* msg) {
  g_last_error = msg;
  return st;
}
}  // namespace spk

namespace {

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      return set_error(SPKADD_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                       __FILE__, __LINE__);                                                    \
    }                                                                                          \
  } while (0)

// ---------------------------------------------------------------------------
// Workspace cache.  Blocks are kept per device and size class (power of two,
// at least 4 KiB).  A freed block is reused at once on the stream that freed it
// (stream order makes that safe) and on another stream once an event recorded at
// free time has completed.
// ---------------------------------------------------------------------------
struct CachedBlock {
  void* ptr;
  hipStream_t stream;
  hipEvent_t done;
};

class WorkspaceCache {
 public:
  static WorkspaceCache& get() {
    static WorkspaceCache* c = new WorkspaceCache();  // never destroyed: outlives static teardown
    return *c;
  }
  static size_t size_class(size_t bytes) {
    size_t s = 4096;
    while (s < bytes) s <<= 1;
    return s;
  }
  hipError_t alloc(void** out, size_t bytes, int dev, hipStream_t stream) {
    const size_t cls = size_class(bytes);
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto& lst = free_[{dev, cls}];
      for (size_t t = 0; t < lst.size(); ++t) {
        CachedBlock b = lst[t];
        bool ok = b.stream == stream;
        if (!ok && b.done) ok = block_idle(b);
        if (ok) {
          if (b.done) (void)hipEventDestroy(b.done);
          lst.erase(lst.begin() + (long)t);
          *out = b.ptr;
          return hipSuccess;
        }
      }
    }
    hipError_t e = hipMalloc(out, cls);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim(dev);
      e = hipMalloc(out, cls);
    }
    return e;
  }
  void release(void* p, size_t bytes, int dev, hipStream_t stream) {
    if (!p) return;
    CachedBlock b{p, stream, nullptr};
    if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) == hipSuccess) {
      if (hipEventRecord(b.done, stream) != hipSuccess) {
        (void)hipEventDestroy(b.done);
        b.done = nullptr;
      }
    } else {
      b.done = nullptr;
    }
    std::lock_guard<std::mutex> lk(mu_);
    free_[{dev, size_class(bytes)}].push_back(b);
  }
  // Frees every cached block of the device whose last use has completed.
  void trim(int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : free_) {
      if (kv.first.first != dev) continue;
      auto& lst = kv.second;
      for (size_t t = 0; t < lst.size();) {
        CachedBlock b = lst[t];
        if (!b.done || block_idle(b)) {
          if (b.done) (void)hipEventDestroy(b.done);
          (void)hipFree(b.ptr);
          lst.erase(lst.begin() + (long)t);
        } else {
          ++t;
        }
      }
    }
  }

 private:
  // Whether the work queued before a block's release has completed.  A query leaves
  // its status in the thread's last-error state (also "not ready"), which is cleared
  // here so that later launch checks see only their own errors.  An event the runtime
  // will not query (one recorded while a graph capture was in progress on another
  // thread) is judged by its stream instead.
  static bool block_idle(const CachedBlock& b) {
    hipError_t e = hipEventQuery(b.done);
    (void)hipGetLastError();
    if (e == hipSuccess) return true;
    if (e == hipErrorNotReady) return false;
    e = hipStreamQuery(b.stream);
    (void)hipGetLastError();
    return e == hipSuccess;
  }
  std::mutex mu_;
  std::map<std::pair<int, size_t>, std::vector<CachedBlock>> free_;
};

// Pinned host slots for the device -> host copies of the plan summary.  A copy into
// pinned memory is asynchronous (a copy into pageable memory makes the host wait
// on its own), and the host can watch the slot while the copy is queued.  Slots
// come from 64 KiB hipHostMalloc chunks and are kept for the life of the process.
class PinnedPool {
 public:
  static constexpr size_t kSlot = 256;
  static_assert(sizeof(PlanSummary) <= kSlot, "slot size");
  static PinnedPool& get() {
    static PinnedPool* p = new PinnedPool();
    return *p;
  }
  void* take() {
    std::lock_guard<std::mutex> lk(mu_);
    if (free_.empty()) {
      void* chunk = nullptr;
      if (hipHostMalloc(&chunk, 64 * 1024, hipHostMallocPortable) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      for (size_t o = 0; o < 64 * 1024; o += kSlot) free_.push_back((char*)chunk + o);
    }
    void* s = free_.back();
    free_.pop_back();
    return s;
  }
  void give(void* s) {
    if (!s) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(s);
  }

 private:
  std::mutex mu_;
  std::vector<void*> free_;
};

// Events, recycled: timing events for SPKADD_FLAG_TRACE (two hipEventRecord calls
// per traced launch) and plain events for host waits.
class EventPool {
 public:
  static EventPool& get() {
    static EventPool* p = new EventPool(0u);
    return *p;
  }
  static EventPool& plain() {
    static EventPool* p = new EventPool(hipEventDisableTiming);
    return *p;
  }
  explicit EventPool(unsigned flags) : flags_(flags) {}
  hipEvent_t take() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!free_.empty()) {
        hipEvent_t e = free_.back();
        free_.pop_back();
        return e;
      }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, flags_) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  void give(hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(e);
  }

 private:
  unsigned flags_;
  std::mutex mu_;
  std::vector<hipEvent_t> free_;
};

struct TraceRec {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace

struct spkadd_plan_s {
  int device = 0;
  int m = 0, n = 0, k = 0;
  spkadd_dtype dtype = SPKADD_F32;
  spkadd_opts opts{};
  PlanParams pp{};
  int alpha_sym_q = 0, alpha_num_q = 0;
  hipStream_t last_stream = nullptr;
  bool failed = false;

  struct Alloc {
    void* p;
    size_t bytes;
  };
  std::vector<Alloc> allocs;

  // pointer tables (device)
  const int** d_cp = nullptr;
  const int** d_ri = nullptr;
  const void** d_va = nullptr;
  // per-column data
  int* d_u = nullptr;
  unsigned char* d_bin = nullptr;
  int* d_colcnt = nullptr;
  int* d_hist = nullptr;
  int* d_binoff = nullptr;
  int* d_list = nullptr;
  PlanSummary* d_sum = nullptr;
  PlanSummary* h_sum = nullptr;  // pinned slot
  hipEvent_t ev_sum = nullptr;   // recorded after each summary copy
  int bin_count[NBINS] = {0};
  int binoff[NBINS + 1] = {0};
  // windows
  int n_wcols = 0, n_windows = 0, levels = 0;
  int max_span = 0;  // widest window (rows)
  int* d_wfirst = nullptr;
  int* d_win_c = nullptr;
  int* d_brow = nullptr;
  int* d_bcol = nullptr;
  int* d_bpos = nullptr;
  int* d_cntin = nullptr;
  int* d_win_cnt = nullptr;
  int* d_win_off = nullptr;
  int4* d_wrec = nullptr;
  // unsorted input: the window columns' entries in one bucket per window
  bool unsorted_in = false;
  long long u_total = 0;           // entries in the buckets
  int* d_ubrows = nullptr;         // bucket rows
  long long* d_ubsrc = nullptr;    // (input << 32 | position) of each bucket entry
  void* d_ubvals = nullptr;        // bucket values, gathered by each numeric pass
  int* d_ubpos = nullptr;          // bucket boundaries, in the one-input layout of bpos
  const void** d_utab = nullptr;   // [0]: bucket rows, [1]: bucket values (one-input pointer tables)
  int n_cu = 256;
  void* d_dummy = nullptr;
  // scan
  void* d_scan_tmp = nullptr;
  // table sizes per bin
  int ts_sym[NBINS] = {0}, ts_num[NBINS] = {0};
  // symbolic results
  int32_t* colptr_c = nullptr;
  int64_t nnz_c = -1;
  bool sym_done = false;
  // the plan's summary copy is queued but not yet waited for (spkadd_symbolic waits)
  bool pending = false;
  hipStream_t plan_stream = nullptr;
  // trace
  std::vector<TraceRec> trace;
  // region mode (the no-allocation entry point): every workspace array is carved
  // from one caller-given device region, never returned, and the summaries are read
  // into this pageable host copy after a wait on the stream
  bool region_mode = false;
  char* region = nullptr;
  size_t region_bytes = 0, region_used = 0;
  PlanSummary h_sum_local{};
  hipStream_t sum_stream = nullptr;

  template <typename T>
  spkadd_status alloc(T** out, size_t count, hipStream_t s) {
    const size_t bytes = (count ? count : 1) * sizeof(T);
    if (region_mode) {
      const size_t off = (region_used + 255) & ~(size_t)255;
      if (off + bytes > region_bytes)
        return set_error(SPKADD_ERR_UNSUPPORTED,
                         "the inputs need more than the %zu bytes of device workspace available here "
                         "(%zu more requested with %zu in use)",
                         region_bytes, bytes, region_used);
      region_used = off + bytes;
      *out = (T*)(region + off);
      return SPKADD_OK;
    }
    void* p = nullptr;
    hipError_t e = WorkspaceCache::get().alloc(&p, bytes, device, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_error(SPKADD_ERR_OOM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    allocs.push_back({p, bytes});
    *out = (T*)p;
    return SPKADD_OK;
  }
  void release(void* p, hipStream_t s) {
    for (size_t t = 0; t < allocs.size(); ++t) {
      if (allocs[t].p == p) {
        WorkspaceCache::get().release(p, allocs[t].bytes, device, s);
        allocs.erase(allocs.begin() + (long)t);
        return;
      }
    }
  }
};

namespace {

bool tracing(const spkadd_plan_s* p, bool numeric) {
  return (p->opts.flags & SPKADD_FLAG_TRACE) != 0 || (numeric && (p->opts.flags & SPKADD_FLAG_TRACE_NUMERIC) != 0);
}

struct TraceScope {
  spkadd_plan_s* p;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  TraceScope(spkadd_plan_s* p_, const char* n, hipStream_t s_, bool numeric = false) : p(p_), name(n), s(s_) {
    if (!tracing(p, numeric)) return;
    a = EventPool::get().take();
    if (a && hipEventRecord(a, s) != hipSuccess) {
      (void)hipGetLastError();
      EventPool::get().give(a);
      a = nullptr;
    }
  }
  ~TraceScope() {
    if (!a) return;
    hipEvent_t b = EventPool::get().take();
    if (b && hipEventRecord(b, s) == hipSuccess) {
      p->trace.push_back({name, a, b});
    } else {
      (void)hipGetLastError();
      EventPool::get().give(a);
      EventPool::get().give(b);
    }
  }
};

void clear_trace(spkadd_plan_s* p) {
  for (auto& t : p->trace) {
    EventPool::get().give(t.a);
    EventPool::get().give(t.b);
  }
  p->trace.clear();
}

constexpr int kDefaultCapF32 = 3072;
constexpr int kDefaultCapF64 = 2048;
constexpr int kMaxCap = 8192;
constexpr float kDefaultAlphaSym = 0.5f;
constexpr float kDefaultAlphaNum = 0.5f;
constexpr float kDefaultFill = 0.75f;
constexpr int kOrderedWaveCap = 1024;  // output entries of a wave-bin column (u_j <= 1024)

int ktop_of(int k) {
  if (k <= 1) return 0;
  int t = 1;
  while (t * 2 <= k - 1) t *= 2;
  return t;
}

bool layout_bin(const spkadd_plan_s* p, int b, bool numeric, KArgs& a);
bool wg_bitmap_bin(const spkadd_plan_s* p, int b);
void wg_bitmap_layout(const spkadd_plan_s* p, int b, bool numeric, KArgs& a, bool worst);

spkadd_status check_lds(spkadd_plan_s* p) {
  const int lmax = max_lds_bytes();
  for (int b = BIN_W1; b < NBINS; ++b) {
    const int cnt = b == BIN_WIN ? p->n_windows : p->bin_count[b];
    if (cnt == 0) continue;
    for (int numeric = 0; numeric < 2; ++numeric) {
      KArgs a{};
      const bool pipe = layout_bin(p, b, numeric != 0, a);
      long long bytes = (long long)a.slice_bytes * (pipe ? PIPE_WAVES_PER_BLOCK : bin_units_per_block(b));
      if (wg_bitmap_bin(p, b)) {
        KArgs ab{};
        wg_bitmap_layout(p, b, numeric != 0, ab, true);
        if (ab.slice_bytes > bytes) bytes = ab.slice_bytes;
      }
      if (bytes > lmax)
        return set_error(SPKADD_ERR_UNSUPPORTED,
                         "bin %d needs %lld bytes of LDS (k=%d, table %d slots); the device has %d", b, bytes, p->k,
                         numeric ? p->ts_num[b] : p->ts_sym[b], lmax);
    }
  }
  return SPKADD_OK;
}

KArgs base_args(const spkadd_plan_s* p) {
  KArgs a{};
  a.cp = p->d_cp;
  a.ri = p->d_ri;
  a.va = p->d_va;
  a.m = p->m;
  a.n = p->n;
  a.k = p->k;
  a.ktop = ktop_of(p->k);
  a.hash_mode = p->opts.hash_mode;
  a.colcnt = p->d_colcnt;
  a.wcols = p->d_list + p->binoff[BIN_WIN];
  a.win_c = p->d_win_c;
  a.brow = p->d_brow;
  a.wrec = p->d_wrec;
  a.bpos = p->d_bpos;
  a.cntin = p->d_cntin;
  a.win_cnt = p->d_win_cnt;
  a.win_off = p->d_win_off;
  a.err = &p->d_sum->err;
  a.dummy = p->d_dummy;
  a.upw = 1;
  return a;
}

// The err field never holds this value on the device (it is a small bit mask).  The
// host stores it before queuing a summary copy; the copy overwrites it.
constexpr int kErrSentinel = 0x7fffffff;

// Queues the copy of the device summary into the pinned slot.
spkadd_status copy_summary(spkadd_plan_s* p, hipStream_t s) {
  __atomic_store_n(&p->h_sum->err, kErrSentinel, __ATOMIC_RELAXED);
  HIP_TRY(hipMemcpyAsync(p->h_sum, p->d_sum, sizeof(PlanSummary), hipMemcpyDeviceToHost, s));
  p->sum_stream = s;
  if (!p->region_mode) HIP_TRY(hipEventRecord(p->ev_sum, s));
  return SPKADD_OK;
}

// Waits for the queued summary copy.  The host first watches the slot with no
// runtime calls until the copy has overwritten the sentinel (polling the runtime
// while kernels run slows their dispatch, and a blocking wait sleeps and wakes up
// tens of microseconds late), then polls the copy's event, which completes a few
// microseconds later.  Each stage falls back to a blocking wait after 20 ms.
spkadd_status wait_summary(spkadd_plan_s* p) {
  if (p->region_mode) {  // pageable copy, no event: wait for the stream
    HIP_TRY(hipStreamSynchronize(p->sum_stream));
    return SPKADD_OK;
  }
  using clk = std::chrono::steady_clock;
  const auto limit = std::chrono::milliseconds(20);
  auto t0 = clk::now();
  while (__atomic_load_n(&p->h_sum->err, __ATOMIC_RELAXED) == kErrSentinel)
    if (clk::now() - t0 > limit) break;
  t0 = clk::now();
  for (;;) {
    const hipError_t e = hipEventQuery(p->ev_sum);
    if (e == hipSuccess) return SPKADD_OK;
    if (e != hipErrorNotReady) return set_error(SPKADD_ERR_HIP, "summary copy: %s", hipGetErrorString(e));
    if (clk::now() - t0 > limit) break;
  }
  (void)hipGetLastError();  // the not-ready status of the polls
  HIP_TRY(hipEventSynchronize(p->ev_sum));
  return SPKADD_OK;
}

spkadd_status sync_summary(spkadd_plan_s* p, hipStream_t s) {
  spkadd_status st = copy_summary(p, s);
  return st ? st : wait_summary(p);
}

spkadd_status check_device_err(spkadd_plan_s* p) {
  const int e = p->h_sum->err;
  if (e & ERR_INPUT) return set_error(SPKADD_ERR_INVALID, "input validation failed (colptr, row range or order)");
  if (e & ERR_OVERFLOW) return set_error(SPKADD_ERR_OVERFLOW, "a count exceeds INT32_MAX");
  if (e & (ERR_PROBE | ERR_COUNT)) {
    p->failed = true;
    return set_error(SPKADD_ERR_HIP, "internal error: device flags 0x%x (table sizing)", e);
  }
  return SPKADD_OK;
}

// Builds the row windows of the window columns: equal row ranges first (the
// paper's split), then windows holding more than cap_in input entries over more
// than cap_in rows are cut again until none is left.
spkadd_status build_windows(spkadd_plan_s* p, hipStream_t s) {
  spkadd_status st;
  const int nwc = p->n_wcols, k = p->k;
  int W = p->n_windows;
  if ((st = p->alloc(&p->d_win_c, W, s))) return st;
  if ((st = p->alloc(&p->d_brow, (size_t)W + nwc, s))) return st;
  if ((st = p->alloc(&p->d_bcol, (size_t)W + nwc, s))) return st;
  if ((st = p->alloc(&p->d_bpos, ((size_t)W + nwc) * k, s))) return st;
  if ((st = p->alloc(&p->d_cntin, W, s))) return st;
  int* d_q = nullptr;
  if ((st = p->alloc(&d_q, W, s))) return st;
  const int* wcols = p->d_list + p->binoff[BIN_WIN];
  int* d_wlin = nullptr;  // columns of the ordered pass
  if ((st = p->alloc(&d_wlin, nwc, s))) return st;
  {
    TraceScope t(p, "win_fill", s);
    launch_win_fill(p->pp, p->d_cp, p->d_ri, wcols, p->d_u, nwc, p->d_wfirst, p->d_win_c, p->d_brow, p->d_bcol,
                    d_wlin, s);
  }
  // work units of the pass over the columns' entries: chunks of each column
  int *d_nch = nullptr, *d_chfirst = nullptr, *d_chcol = nullptr;
  void* chtmp = nullptr;
  if ((st = p->alloc(&d_nch, nwc, s))) return st;
  if ((st = p->alloc(&d_chfirst, (size_t)nwc + 1, s))) return st;
  if ((st = p->alloc((char**)&chtmp, scan_tmp_bytes(nwc), s))) return st;
  launch_uwin_chunks(p->pp, nwc, wcols, p->d_u, WIN_LOC_CHUNK, d_wlin, d_nch, s);
  launch_scan(d_nch, nwc, d_chfirst, &p->d_sum->total, &p->d_sum->err, chtmp, s);
  if ((st = sync_summary(p, s))) return st;
  if ((st = check_device_err(p))) return st;
  const long long nchunks = p->h_sum->total;
  if (nchunks > INT_MAX / 2) return set_error(SPKADD_ERR_OVERFLOW, "too many window chunks (%lld)", nchunks);
  int* d_bpos_t = nullptr;
  if ((st = p->alloc(&d_chcol, (size_t)nchunks, s))) return st;
  if ((st = p->alloc(&d_bpos_t, ((size_t)W + nwc) * k, s))) return st;
  launch_uwin_chfill(nwc, d_chfirst, d_chcol, s);
  {
    TraceScope t(p, "win_search", s);
    launch_win_search(p->pp, p->d_cp, p->d_ri, wcols, p->d_wfirst, d_wlin, nwc, p->d_brow, p->d_bcol, W + nwc,
                      (int)nchunks, d_chfirst, d_chcol, d_bpos_t, p->d_bpos, s);
  }
  p->release(d_nch, s);
  p->release(d_chfirst, s);
  p->release(chtmp, s);
  p->release(d_chcol, s);
  p->release(d_bpos_t, s);
  p->release(d_wlin, s);
  HIP_TRY(hipMemsetAsync(&p->d_sum->pad, 0, 2 * sizeof(int), s));  // pad and max_span
  {
    TraceScope t(p, "win_count", s);
    launch_win_count(p->pp, W, p->d_win_c, p->d_brow, p->d_bpos, p->d_cntin, d_q, p->d_sum, s);
  }
  HIP_TRY(hipGetLastError());
  if ((st = sync_summary(p, s))) return st;
  p->levels = 0;
  while (p->h_sum->pad > 0) {
    if (++p->levels > 64) return set_error(SPKADD_ERR_HIP, "window refinement did not converge");
    // new window numbering: exclusive scan of the pieces per window
    int* d_newfirst = nullptr;
    void* tmp = nullptr;
    if ((st = p->alloc(&d_newfirst, (size_t)W + 1, s))) return st;
    if ((st = p->alloc((char**)&tmp, scan_tmp_bytes(W), s))) return st;
    launch_scan(d_q, W, d_newfirst, &p->d_sum->total, &p->d_sum->err, tmp, s);
    if ((st = sync_summary(p, s))) return st;
    const long long total = p->h_sum->total;
    if (total > INT_MAX / 2 || (total + nwc) * (long long)k > (long long)INT_MAX * 64)
      return set_error(SPKADD_ERR_OVERFLOW, "too many row windows (%lld)", total);
    const int W2 = (int)total;
    int *win_c2, *brow2, *bcol2, *bpos2, *bpar, *bpiece, *wfirst2, *cntin2, *q2;
    if ((st = p->alloc(&win_c2, W2, s))) return st;
    if ((st = p->alloc(&brow2, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&bcol2, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&bpos2, ((size_t)W2 + nwc) * k, s))) return st;
    if ((st = p->alloc(&bpar, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&bpiece, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&wfirst2, (size_t)nwc + 1, s))) return st;
    if ((st = p->alloc(&cntin2, W2, s))) return st;
    if ((st = p->alloc(&q2, W2, s))) return st;
    {
      TraceScope t(p, "win_refine_fill", s);
      launch_win_refine_fill(p->pp, W, nwc, p->d_win_c, p->d_wfirst, d_q, d_newfirst, p->d_brow, p->d_ri,
                             p->d_bpos, win_c2, brow2, bcol2, bpar, bpiece, wfirst2, s);
    }
    {
      TraceScope t(p, "win_refine_search", s);
      launch_win_refine_search(p->pp, p->d_ri, W2 + nwc, bcol2, brow2, bpar, bpiece, d_q, p->d_bpos, bpos2, s);
    }
    HIP_TRY(hipMemsetAsync(&p->d_sum->pad, 0, 2 * sizeof(int), s));  // pad and max_span
    {
      TraceScope t(p, "win_count", s);
      launch_win_count(p->pp, W2, win_c2, brow2, bpos2, cntin2, q2, p->d_sum, s);
    }
    HIP_TRY(hipGetLastError());
    if ((st = sync_summary(p, s))) return st;
    // retire the previous level
    p->release(p->d_win_c, s);
    p->release(p->d_brow, s);
    p->release(p->d_bcol, s);
    p->release(p->d_bpos, s);
    p->release(p->d_cntin, s);
    p->release(d_q, s);
    p->release(p->d_wfirst, s);
    p->release(d_newfirst, s);
    p->release(tmp, s);
    p->release(bpar, s);
    p->release(bpiece, s);
    p->d_win_c = win_c2;
    p->d_brow = brow2;
    p->d_bcol = bcol2;
    p->d_bpos = bpos2;
    p->d_cntin = cntin2;
    p->d_wfirst = wfirst2;
    d_q = q2;
    W = W2;
  }
  p->release(d_q, s);
  p->n_windows = W;
  p->max_span = p->h_sum->max_span;  // of the last level counted (the final windows)
  if ((st = p->alloc(&p->d_win_cnt, W, s))) return st;
  if ((st = p->alloc(&p->d_win_off, W, s))) return st;
  if ((st = p->alloc(&p->d_wrec, W, s))) return st;
  {
    TraceScope t(p, "win_records", s);
    launch_win_records(W, wcols, p->d_win_c, p->d_brow, p->d_wrec, s);
  }
  HIP_TRY(hipGetLastError());
  return SPKADD_OK;
}


// Row windows of unsorted input columns: the same splits as build_windows, with each
// level's window counts from a histogram of the column's rows against its window
// boundaries (no binary search, which needs sorted columns); the final windows' entries
// are then partitioned into one bucket per window.
spkadd_status build_windows_unsorted(spkadd_plan_s* p, hipStream_t s) {
  spkadd_status st;
  const int nwc = p->n_wcols;
  int W = p->n_windows;
  if ((st = p->alloc(&p->d_win_c, W, s))) return st;
  if ((st = p->alloc(&p->d_brow, (size_t)W + nwc, s))) return st;
  if ((st = p->alloc(&p->d_bcol, (size_t)W + nwc, s))) return st;
  if ((st = p->alloc(&p->d_cntin, W, s))) return st;
  int* d_q = nullptr;
  if ((st = p->alloc(&d_q, W, s))) return st;
  const int* wcols = p->d_list + p->binoff[BIN_WIN];
  {
    TraceScope t(p, "win_fill", s);
    launch_win_fill(p->pp, p->d_cp, p->d_ri, wcols, p->d_u, nwc, p->d_wfirst, p->d_win_c, p->d_brow, p->d_bcol,
                    nullptr, s);
  }
  // work units of the passes over the columns' entries: chunks of each column
  int *d_nch = nullptr, *d_chfirst = nullptr, *d_chcol = nullptr;
  void* chtmp = nullptr;
  if ((st = p->alloc(&d_nch, nwc, s))) return st;
  if ((st = p->alloc(&d_chfirst, (size_t)nwc + 1, s))) return st;
  if ((st = p->alloc((char**)&chtmp, scan_tmp_bytes(nwc), s))) return st;
  launch_uwin_chunks(p->pp, nwc, wcols, p->d_u, WIN_CHUNK, nullptr, d_nch, s);
  launch_scan(d_nch, nwc, d_chfirst, &p->d_sum->total, &p->d_sum->err, chtmp, s);
  if ((st = sync_summary(p, s))) return st;
  if ((st = check_device_err(p))) return st;
  const long long nchunks = p->h_sum->total;
  if (nchunks > INT_MAX / 2) return set_error(SPKADD_ERR_OVERFLOW, "too many window chunks (%lld)", nchunks);
  if ((st = p->alloc(&d_chcol, (size_t)nchunks, s))) return st;
  launch_uwin_chfill(nwc, d_chfirst, d_chcol, s);
  p->levels = 0;
  for (;;) {
    HIP_TRY(hipMemsetAsync(p->d_cntin, 0, (size_t)W * sizeof(int), s));
    {
      TraceScope t(p, "uwin_hist", s);
      launch_uwin_hist(p->pp, p->d_cp, p->d_ri, (int)nchunks, wcols, p->d_wfirst, p->d_brow, d_chfirst, d_chcol,
                       p->d_cntin, s);
    }
    HIP_TRY(hipMemsetAsync(&p->d_sum->pad, 0, 2 * sizeof(int), s));  // pad and max_span
    {
      TraceScope t(p, "win_count", s);
      launch_win_count(p->pp, W, p->d_win_c, p->d_brow, nullptr, p->d_cntin, d_q, p->d_sum, s);
    }
    HIP_TRY(hipGetLastError());
    if ((st = sync_summary(p, s))) return st;
    if (p->h_sum->pad == 0) break;
    if (++p->levels > 64) return set_error(SPKADD_ERR_HIP, "window refinement did not converge");
    int* d_newfirst = nullptr;
    void* tmp = nullptr;
    if ((st = p->alloc(&d_newfirst, (size_t)W + 1, s))) return st;
    if ((st = p->alloc((char**)&tmp, scan_tmp_bytes(W), s))) return st;
    launch_scan(d_q, W, d_newfirst, &p->d_sum->total, &p->d_sum->err, tmp, s);
    if ((st = sync_summary(p, s))) return st;
    const long long total = p->h_sum->total;
    if (total > INT_MAX / 2) return set_error(SPKADD_ERR_OVERFLOW, "too many row windows (%lld)", total);
    const int W2 = (int)total;
    int *win_c2, *brow2, *bcol2, *bpar, *bpiece, *wfirst2, *cntin2, *q2;
    if ((st = p->alloc(&win_c2, W2, s))) return st;
    if ((st = p->alloc(&brow2, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&bcol2, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&bpar, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&bpiece, (size_t)W2 + nwc, s))) return st;
    if ((st = p->alloc(&wfirst2, (size_t)nwc + 1, s))) return st;
    if ((st = p->alloc(&cntin2, W2, s))) return st;
    if ((st = p->alloc(&q2, W2, s))) return st;
    {
      TraceScope t(p, "win_refine_fill", s);
      launch_win_refine_fill(p->pp, W, nwc, p->d_win_c, p->d_wfirst, d_q, d_newfirst, p->d_brow, p->d_ri,
                             nullptr, win_c2, brow2, bcol2, bpar, bpiece, wfirst2, s);
    }
    for (void* x : {(void*)p->d_win_c, (void*)p->d_brow, (void*)p->d_bcol, (void*)p->d_cntin, (void*)d_q,
                    (void*)p->d_wfirst, (void*)d_newfirst, tmp, (void*)bpar, (void*)bpiece})
      p->release(x, s);
    p->d_win_c = win_c2;
    p->d_brow = brow2;
    p->d_bcol = bcol2;
    p->d_cntin = cntin2;
    p->d_wfirst = wfirst2;
    d_q = q2;
    W = W2;
  }
  p->release(d_q, s);
  p->n_windows = W;
  p->max_span = p->h_sum->max_span;
  // buckets: offsets, boundaries in the one-input layout, then the partition
  int* d_boff = nullptr;
  int* d_gcur = nullptr;
  void* tmp = nullptr;
  if ((st = p->alloc(&d_boff, (size_t)W + 1, s))) return st;
  if ((st = p->alloc((char**)&tmp, scan_tmp_bytes(W), s))) return st;
  launch_scan(p->d_cntin, W, d_boff, &p->d_sum->total, &p->d_sum->err, tmp, s);
  if ((st = sync_summary(p, s))) return st;
  if ((st = check_device_err(p))) return st;
  p->u_total = p->h_sum->total;
  const int vb = p->dtype == SPKADD_F64 ? 8 : 4;
  if ((st = p->alloc(&p->d_ubpos, (size_t)W + nwc, s))) return st;
  if ((st = p->alloc(&p->d_ubrows, (size_t)p->u_total, s))) return st;
  if ((st = p->alloc(&p->d_ubsrc, (size_t)p->u_total, s))) return st;
  if ((st = p->alloc((char**)&p->d_ubvals, (size_t)p->u_total * vb, s))) return st;
  if ((st = p->alloc(&p->d_utab, 2, s))) return st;
  if ((st = p->alloc(&d_gcur, W, s))) return st;
  launch_uwin_bpos(W, p->d_win_c, p->d_wfirst, d_boff, p->d_ubpos, s);
  HIP_TRY(hipMemcpyAsync(d_gcur, d_boff, (size_t)W * sizeof(int), hipMemcpyDeviceToDevice, s));
  {
    TraceScope t(p, "uwin_scatter", s);
    launch_uwin_scatter(p->pp, p->d_cp, p->d_ri, (int)nchunks, wcols, p->d_wfirst, p->d_brow, d_chfirst, d_chcol,
                        d_gcur, p->d_ubrows, p->d_ubsrc, s);
  }
  const void* tab[2] = {p->d_ubrows, p->d_ubvals};
  launch_put_ptrs(tab, 2, p->d_utab, nullptr, nullptr, s);
  HIP_TRY(hipGetLastError());
  for (void* x : {tmp, (void*)d_boff, (void*)d_gcur, (void*)d_nch, (void*)d_chfirst, (void*)d_chcol, chtmp})
    p->release(x, s);
  if ((st = p->alloc(&p->d_win_cnt, W, s))) return st;
  if ((st = p->alloc(&p->d_win_off, W, s))) return st;
  if ((st = p->alloc(&p->d_wrec, W, s))) return st;
  {
    TraceScope t(p, "win_records", s);
    launch_win_records(W, wcols, p->d_win_c, p->d_brow, p->d_wrec, s);
  }
  HIP_TRY(hipGetLastError());
  return SPKADD_OK;
}

bool is_wave(int b) { return b >= BIN_W1 && b <= BIN_W16; }

// Bitmap rows (of 256 words) for a wave bin, or 0 for hash tables.
int bitmap_rows(const spkadd_plan_s* p, int b) {
  if (!is_wave(b) || p->opts.accum_mode == SPKADD_ACCUM_HASH) return 0;
  const long long nq = ((long long)p->m + 8191) / 8192;
  if (nq < 1 || nq > 16) return 0;
  if (p->opts.accum_mode == SPKADD_ACCUM_BITMAP) return (int)nq;
  const float ratio = p->opts.bitmap_ratio > 0 ? p->opts.bitmap_ratio : 1.0f;
  return nq <= ratio * wave_bin_E(b) ? (int)nq : 0;
}

// LDS layout of bin b for a phase; returns whether the pipelined wave kernel runs it.
bool layout_bin(const spkadd_plan_s* p, int b, bool numeric, KArgs& a) {
  const int vb = p->dtype == SPKADD_F64 ? 8 : 4;
  const int ts = numeric ? p->ts_num[b] : p->ts_sym[b];
  if (is_wave(b) && wave_pipe_ok(p->k, p->alpha_num_q)) {
    lds_layout_pipe(b, numeric, vb, ts, bitmap_rows(p, b), a);
    return true;
  }
  lds_layout(b, numeric, vb, p->k, ts, a);
  a.bm_nq = 0;
  return false;
}

// Workgroup units (G1, G2, windows) narrow enough for a bitmap over their row range
// use it, unless hash tables are asked for (accum_mode, or the degenerate-hash test
// hook, which is about the tables).
bool wg_bitmap_bin(const spkadd_plan_s* p, int b) {
  if (b != BIN_G1 && b != BIN_G2 && b != BIN_WIN) return false;
  if (p->opts.accum_mode == SPKADD_ACCUM_HASH || p->opts.hash_mode != 0) return false;
  return b == BIN_WIN || p->m <= bitmap_wg_span_max();
}

// The bitmap is sized for the widest unit of the bin (rounded up to a power of two,
// at most bitmap_wg_span_max()); worst: the largest it can be (before the windows exist).
void wg_bitmap_layout(const spkadd_plan_s* p, int b, bool numeric, KArgs& a, bool worst = false) {
  const int cap = bitmap_wg_span_max();
  const long long need = worst ? cap : b == BIN_WIN ? p->max_span : p->m;
  int span = 1024;
  while (span < need && span < cap) span <<= 1;
  const int vb = p->dtype == SPKADD_F64 ? 8 : 4, regs = bitmap_wg_regs(b);
  lds_layout_bitmap_wg(numeric, vb, p->k, span, p->pp.cap_in, regs, false, 2, a);
  if (!numeric) return;
  // groups of four words halve the prefix; worth their costlier ranks only where that
  // lets another workgroup reside (resident waves per CU are capped at 32)
  KArgs a4 = a;
  lds_layout_bitmap_wg(numeric, vb, p->k, span, p->pp.cap_in, regs, false, 4, a4);
  const int waves = (b == BIN_G1 ? G1_THREADS : G2_THREADS) / 64, lmax = max_lds_bytes();
  auto resident = [&](const KArgs& x) {
    const int by_lds = lmax / (x.slice_bytes > 0 ? x.slice_bytes : 1), by_waves = 32 / waves;
    return by_lds < by_waves ? by_lds : by_waves;
  };
  if (resident(a4) > resident(a)) a = a4;
}

// Launches the symbolic or numeric kernel of bin b.
hipError_t launch_bin(spkadd_plan_s* p, int b, bool numeric, KArgs& a_in, hipStream_t s) {
  const int cnt = b == BIN_WIN ? p->n_windows : p->bin_count[b];
  if (cnt == 0) return hipSuccess;
  KArgs a = a_in;
  if (b == BIN_WIN && p->unsorted_in) {  // the buckets: one input, boundaries in bpos layout
    a.k = 1;
    a.ktop = 0;
    a.ri = (const int* const*)p->d_utab;
    a.va = (const void* const*)(p->d_utab + 1);
    a.bpos = p->d_ubpos;
  }
  const bool f64 = p->dtype == SPKADD_F64;
  const int* list = b == BIN_WIN ? nullptr : p->d_list + p->binoff[b];
  if (wg_bitmap_bin(p, b)) {
    // workgroup bitmap for every unit at most span_max rows wide; the hash kernel
    // takes the wider ones (only windows can be wider)
    KArgs ab = a;
    wg_bitmap_layout(p, b, numeric, ab);
    hipError_t e = launch_bitmap_wg(b, numeric, f64, ab, list, cnt, s);
    if (e != hipSuccess || b != BIN_WIN || p->max_span <= ab.wg_span_max) return e;
    layout_bin(p, b, numeric, a);
    a.wg_span_max = ab.wg_span_max;
    TraceScope t(p, numeric ? "num_window_wide" : "sym_window_wide", s, numeric);
    return launch_hash(b, numeric, f64, a, list, cnt, s);
  }
  if (layout_bin(p, b, numeric, a)) {
    // resident wavefronts per CU: LDS-bound, at most 16 (four per SIMD)
    const int block_lds = a.slice_bytes * PIPE_WAVES_PER_BLOCK;
    int bpc = max_lds_bytes() / block_lds;
    if (bpc > 16 / PIPE_WAVES_PER_BLOCK) bpc = 16 / PIPE_WAVES_PER_BLOCK;
    if (bpc < 1) bpc = 1;
    const long long resident = (long long)p->n_cu * bpc * PIPE_WAVES_PER_BLOCK;
    long long upw = (cnt + resident - 1) / resident;
    a.upw = (int)(upw < 1 ? 1 : upw > 64 ? 64 : upw);
    return launch_wave_pipe(b, numeric, f64, a, list, cnt, s);
  }
  return launch_hash(b, numeric, f64, a, list, cnt, s);
}

// The fused symbolic launch of the wave bins (wave_fused.hip): each bin's accumulator
// and table size, the largest LDS slice of any wave bin, and the grid (resident
// blocks).  False when some wave bin does not take the pipelined kernel or the
// slices do not fit.
bool wave_sym_fused_setup(const spkadd_plan_s* p, KArgs& a, WaveBinTable& t, unsigned& blocks) {
  int slice = 0;
  for (int wi = 0; wi < NWAVE_BINS; ++wi) {
    const int b = BIN_W1 + wi;
    KArgs x{};
    if (!layout_bin(p, b, false, x)) return false;
    t.bm_nq[wi] = x.bm_nq;
    t.ts[wi] = p->ts_sym[b];
    if (x.slice_bytes > slice) slice = x.slice_bytes;
  }
  int bpc = max_lds_bytes() / (slice * PIPE_WAVES_PER_BLOCK);
  if (bpc > 16 / PIPE_WAVES_PER_BLOCK) bpc = 16 / PIPE_WAVES_PER_BLOCK;  // four wavefronts per SIMD
  if (bpc < 1) return false;
  a.slice_bytes = slice;
  blocks = (unsigned)(p->n_cu * bpc);
  return true;
}

spkadd_status plan_finish(spkadd_plan_s* p, hipStream_t stream);

void release_all(spkadd_plan_s* p) {
  if (p->pending) {  // the summary copy into the pinned slot may still be in flight
    if (wait_summary(p) != SPKADD_OK) (void)hipGetLastError();
    p->pending = false;
  }
  hipStream_t s = p->last_stream;
  for (auto& a : p->allocs) WorkspaceCache::get().release(a.p, a.bytes, p->device, s);
  p->allocs.clear();
  if (!p->region_mode) {
    PinnedPool::get().give(p->h_sum);  // every copy into it was waited for
    EventPool::plain().give(p->ev_sum);
  }
  p->h_sum = nullptr;
  p->ev_sum = nullptr;
}

// Argument checks and the planning step into plan p (constructed by the caller, who
// releases it on an error).
spkadd_status plan_build(spkadd_plan_s* p, int32_t m, int32_t n, int32_t k, const int32_t* const* colptr,
                         const int32_t* const* rowidx, spkadd_dtype dtype, const spkadd_opts* opts,
                         hipStream_t stream) {
  if (m < 0 || n < 0 || m == INT_MAX || n == INT_MAX)
    return set_error(SPKADD_ERR_INVALID, "bad shape m=%d n=%d", m, n);
  if (k < 1) return set_error(SPKADD_ERR_INVALID, "k must be >= 1 (got %d)", k);
  if (!colptr || !rowidx) return set_error(SPKADD_ERR_INVALID, "colptr / rowidx pointer arrays are NULL");
  for (int i = 0; i < k; ++i)
    if (!colptr[i]) return set_error(SPKADD_ERR_INVALID, "colptr[%d] is NULL", i);
  if (dtype != SPKADD_F32 && dtype != SPKADD_F64) return set_error(SPKADD_ERR_INVALID, "bad dtype %d", (int)dtype);
  spkadd_opts o;
  spkadd_opts_default(&o);
  if (opts) o = *opts;
  if (o.force_bin < -1 || o.force_bin > 2) return set_error(SPKADD_ERR_INVALID, "bad force_bin %d", o.force_bin);
  if (o.hash_mode < 0 || o.hash_mode > 1) return set_error(SPKADD_ERR_INVALID, "bad hash_mode %d", o.hash_mode);
  if (o.wave_max < 0 || o.wave_max > 1024) return set_error(SPKADD_ERR_INVALID, "wave_max must be in [0, 1024]");
  if (o.window_cap < 0 || o.window_cap > kMaxCap)
    return set_error(SPKADD_ERR_INVALID, "window_cap must be in [0, %d]", kMaxCap);
  if (!(o.load_factor_sym >= 0.f && o.load_factor_sym <= 0.9f))
    return set_error(SPKADD_ERR_INVALID, "load_factor_sym must be in [0, 0.9]");
  if (!(o.load_factor_num >= 0.f && o.load_factor_num <= 0.5f))
    return set_error(SPKADD_ERR_INVALID, "load_factor_num must be in [0, 0.5]");
  if (!(o.window_fill >= 0.f && o.window_fill <= 1.f))
    return set_error(SPKADD_ERR_INVALID, "window_fill must be in [0, 1]");
  if (o.accum_mode < 0 || o.accum_mode > 2) return set_error(SPKADD_ERR_INVALID, "bad accum_mode %d", o.accum_mode);
  if (!(o.bitmap_ratio >= 0.f && o.bitmap_ratio <= 64.f))
    return set_error(SPKADD_ERR_INVALID, "bitmap_ratio must be in [0, 64]");
  if (o.wave_merge < 0 || o.wave_merge > 1) return set_error(SPKADD_ERR_INVALID, "bad wave_merge %d", o.wave_merge);
  if ((o.flags & SPKADD_FLAG_ORDERED) && (o.flags & SPKADD_FLAG_UNSORTED_IN))
    return set_error(SPKADD_ERR_UNSUPPORTED, "SPKADD_FLAG_ORDERED does not take SPKADD_FLAG_UNSORTED_IN");

  auto fail = [](spkadd_status st) { return st; };  // the caller releases the plan
  if (hipGetDevice(&p->device) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(SPKADD_ERR_HIP, "no HIP device");
  }
  p->m = m;
  p->n = n;
  p->k = k;
  p->dtype = dtype;
  p->opts = o;
  p->last_stream = stream;
  const int cap = o.window_cap ? o.window_cap : (dtype == SPKADD_F64 ? kDefaultCapF64 : kDefaultCapF32);
  const float asym = o.load_factor_sym > 0 ? o.load_factor_sym : kDefaultAlphaSym;
  const float anum = o.load_factor_num > 0 ? o.load_factor_num : kDefaultAlphaNum;
  p->alpha_sym_q = alpha_to_q(asym);
  p->alpha_num_q = alpha_to_q(anum);
  p->pp.m = m;
  p->pp.n = n;
  p->pp.k = k;
  p->pp.wave_max = o.wave_max ? o.wave_max : 1024;
  p->pp.cap_in = cap;
  // G1 stages at most 16 numeric table slots per thread; shrink its column limit
  // until its tables fit (small load factors make tables larger).
  int g1 = cap < 2048 ? cap : 2048;
  while (g1 > 64 && table_slots(g1, p->alpha_num_q) > G1_THREADS * 16) g1 -= 64;
  p->pp.g1_max = g1;
  p->pp.force_bin = o.force_bin;
  p->pp.win_fill = o.window_fill > 0 ? o.window_fill : kDefaultFill;
  p->unsorted_in = (o.flags & SPKADD_FLAG_UNSORTED_IN) != 0;
  p->pp.unsorted_in = p->unsorted_in ? 1 : 0;
  // windows no wider than the workgroup bitmap, so that none falls back to hash
  // tables (unless hash tables are asked for)
  p->pp.win_min = 1;
  p->pp.win_span = INT_MAX;
  if (o.accum_mode != SPKADD_ACCUM_HASH && o.hash_mode == 0 && m > bitmap_wg_span_max()) {
    p->pp.win_min = (int)(((long long)m + bitmap_wg_span_max() - 1) / bitmap_wg_span_max());
    p->pp.win_span = bitmap_wg_span_max();
  }
  for (int b = BIN_W1; b <= BIN_W16; ++b) {
    p->ts_sym[b] = table_slots(64 * wave_bin_E(b), p->alpha_sym_q);
    p->ts_num[b] = table_slots(64 * wave_bin_E(b), p->alpha_num_q);
  }
  p->ts_sym[BIN_G1] = table_slots(p->pp.g1_max, p->alpha_sym_q);
  p->ts_num[BIN_G1] = table_slots(p->pp.g1_max, p->alpha_num_q);
  p->ts_sym[BIN_G2] = p->ts_sym[BIN_WIN] = table_slots(cap, p->alpha_sym_q);
  p->ts_num[BIN_G2] = p->ts_num[BIN_WIN] = table_slots(cap, p->alpha_num_q);
  if (p->ts_num[BIN_G1] > G1_THREADS * 16 || p->ts_num[BIN_G2] > G2_THREADS * 32)
    return fail(set_error(SPKADD_ERR_INVALID, "window_cap / load_factor_num give too large numeric tables"));
  if (o.flags & SPKADD_FLAG_ORDERED) {
    const int need = ordered_lds_bytes(k, cap > kOrderedWaveCap ? cap : kOrderedWaveCap, dtype == SPKADD_F64 ? 8 : 4);
    if (need > max_lds_bytes())
      return fail(set_error(SPKADD_ERR_UNSUPPORTED, "SPKADD_FLAG_ORDERED with k=%d needs %d bytes of LDS per unit", k,
                            need));
  }

  spkadd_status st;
  const int nblk = n > 0 ? (n + PLAN_THREADS - 1) / PLAN_THREADS : 1;
  if (p->region_mode) {
    p->h_sum = &p->h_sum_local;
  } else {
    p->h_sum = (PlanSummary*)PinnedPool::get().take();
    if (!p->h_sum) return fail(set_error(SPKADD_ERR_OOM, "pinned host allocation failed"));
    p->ev_sum = EventPool::plain().take();
    if (!p->ev_sum) return fail(set_error(SPKADD_ERR_HIP, "event creation failed"));
  }
  memset(p->h_sum, 0, sizeof(PlanSummary));
  // one workspace block for the fixed per-plan buffers
  {
    size_t off = 0;
    auto carve = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) & ~(size_t)255;
      return o;
    };
    const size_t o_ptrs = carve(3 * (size_t)k * sizeof(void*));
    const size_t o_u = carve((size_t)n * 4), o_bin = carve((size_t)n), o_colcnt = carve((size_t)n * 4);
    const size_t o_hist = carve((size_t)nblk * NBINS * 4), o_binoff = carve((2 * NBINS + 1) * 4);
    const size_t o_list = carve((size_t)n * 4), o_sum = carve(sizeof(PlanSummary));
    const size_t o_wfirst = carve(((size_t)n + 1) * 4), o_scan = carve(scan_tmp_bytes(n));
    const size_t o_dummy = carve(4096);
    char* arena = nullptr;
    if ((st = p->alloc(&arena, off, stream))) return fail(st);
    p->d_cp = (const int**)(arena + o_ptrs);
    p->d_ri = p->d_cp + k;
    p->d_va = (const void**)(p->d_ri + k);
    p->d_u = (int*)(arena + o_u);
    p->d_bin = (unsigned char*)(arena + o_bin);
    p->d_colcnt = (int*)(arena + o_colcnt);
    p->d_hist = (int*)(arena + o_hist);
    p->d_binoff = (int*)(arena + o_binoff);
    p->d_list = (int*)(arena + o_list);
    p->d_sum = (PlanSummary*)(arena + o_sum);
    p->d_wfirst = (int*)(arena + o_wfirst);
    p->d_scan_tmp = arena + o_scan;
    p->d_dummy = arena + o_dummy;
  }
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
      p->n_cu = cus;
  }

  auto hipfail = [&](hipError_t e, const char* what) {
    (void)hipGetLastError();
    return fail(set_error(SPKADD_ERR_HIP, "%s: %s", what, hipGetErrorString(e)));
  };
  hipError_t e;
  {
    TraceScope t(p, "put_ptrs", stream);
    if (p->region_mode) {  // (two launches, no host copy of the pointer arrays)
      launch_put_ptrs((const void* const*)colptr, k, (const void**)p->d_cp, p->d_sum, p->d_dummy, stream);
      launch_put_ptrs((const void* const*)rowidx, k, (const void**)p->d_ri, nullptr, nullptr, stream);
    } else {
      std::vector<const void*> host_ptrs(2 * (size_t)k);
      for (int i = 0; i < k; ++i) {
        host_ptrs[i] = colptr[i];
        host_ptrs[k + i] = rowidx[i];
      }
      launch_put_ptrs(host_ptrs.data(), 2 * k, (const void**)p->d_cp, p->d_sum, p->d_dummy, stream);
    }
  }
  if (o.flags & SPKADD_FLAG_VALIDATE) {
    TraceScope t(p, "validate", stream);
    launch_validate(p->pp, p->d_cp, p->d_ri, p->d_sum, stream);
  }
  {
    TraceScope t(p, "bounds", stream);
    launch_bounds(p->pp, p->d_cp, p->d_ri, p->d_u, p->d_bin, p->d_colcnt, p->d_hist, p->d_sum, stream);
  }
  {
    TraceScope t(p, "bin_scan", stream);
    launch_bin_scan(nblk, o.wave_merge == 0, p->d_hist, p->d_binoff, p->d_sum, stream);
  }
  if ((e = hipGetLastError())) return hipfail(e, "plan kernels");
  // Deferred wait: the column lists are built, then the summary copy is queued, and
  // spkadd_symbolic waits for it once the symbolic pass of the wave bins (which needs
  // no bin count on the host) is running.  The plan waits here when it validates its
  // inputs (the validation errors are the plan's), when an input has no row array,
  // in region mode (pageable summaries) and when the wave bins do not take the
  // pipelined kernels.
  bool defer = !p->region_mode && !(o.flags & SPKADD_FLAG_VALIDATE) && wave_pipe_ok(k, p->alpha_num_q);
  for (int i = 0; i < k && defer; ++i) defer = rowidx[i] != nullptr;
  if (defer) {
    KArgs fa{};
    WaveBinTable ft{};
    unsigned fb = 0;
    defer = wave_sym_fused_setup(p, fa, ft, fb);
  }
  if (defer) {
    {
      TraceScope t(p, "bin_scatter", stream);
      launch_bin_scatter(p->pp, p->d_bin, p->d_hist, p->d_binoff, p->d_list, stream);
    }
    if ((e = hipGetLastError())) return hipfail(e, "plan kernels");
    if ((st = copy_summary(p, stream))) return fail(st);  // (its event also covers the column lists)
    p->pending = true;
    p->plan_stream = stream;
    return SPKADD_OK;
  }
  // the host needs the bin counts; the column lists are built while it waits
  if ((st = copy_summary(p, stream))) return fail(st);
  {
    TraceScope t(p, "bin_scatter", stream);
    launch_bin_scatter(p->pp, p->d_bin, p->d_hist, p->d_binoff, p->d_list, stream);
  }
  if ((e = hipGetLastError())) return hipfail(e, "plan kernels");
  return plan_finish(p, stream);
}

// The part of the planning step after the bin counts are on the host: bin offsets,
// LDS checks and the row windows.
spkadd_status plan_finish(spkadd_plan_s* p, hipStream_t stream) {
  auto fail = [](spkadd_status st) { return st; };
  auto hipfail = [&](hipError_t e, const char* what) {
    (void)hipGetLastError();
    return fail(set_error(SPKADD_ERR_HIP, "%s: %s", what, hipGetErrorString(e)));
  };
  hipError_t e;
  spkadd_status st;
  if ((st = wait_summary(p))) return fail(st);  // (still pending: spkadd_free waits again)
  p->pending = false;
  if ((st = check_device_err(p))) return fail(st);
  int acc = 0;
  for (int b = 0; b < NBINS; ++b) {
    p->bin_count[b] = p->h_sum->bin_count[b];
    p->binoff[b] = acc;
    acc += p->bin_count[b];
  }
  p->binoff[NBINS] = acc;
  p->n_wcols = p->bin_count[BIN_WIN];
  p->n_windows = 0;
  if ((st = check_lds(p))) return fail(st);
  if (p->n_wcols > 0) {
    {
      TraceScope t(p, "win_scan", stream);
      launch_win_scan(p->pp, p->d_list, p->d_binoff, p->d_u, p->d_wfirst, p->d_sum, stream);
    }
    if ((e = hipGetLastError())) return hipfail(e, "plan kernels");
    if ((st = sync_summary(p, stream))) return fail(st);
    if ((st = check_device_err(p))) return fail(st);
    p->n_windows = p->h_sum->n_windows;
    if ((st = check_lds(p))) return fail(st);
    if ((st = (p->unsorted_in ? build_windows_unsorted(p, stream) : build_windows(p, stream)))) return fail(st);
    if ((st = check_device_err(p))) return fail(st);
  }
  return SPKADD_OK;
}

}  // namespace

extern "C" {

void spkadd_opts_default(spkadd_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->force_bin = SPKADD_BIN_AUTO;
}

const char* spkadd_last_error(void) { return g_last_error.c_str(); }

spkadd_status spkadd_plan(spkadd_plan_t* out, int32_t m, int32_t n, int32_t k, const int32_t* const* colptr,
                          const int32_t* const* rowidx, spkadd_dtype dtype, const spkadd_opts* opts,
                          hipStream_t stream) {
  g_last_error.clear();
  (void)hipGetLastError();  // a stale status of the caller's earlier HIP calls
  if (!out) return set_error(SPKADD_ERR_INVALID, "out is NULL");
  *out = nullptr;
  auto* p = new (std::nothrow) spkadd_plan_s();
  if (!p) return set_error(SPKADD_ERR_OOM, "host allocation failed");
  const spkadd_status st = plan_build(p, m, n, k, colptr, rowidx, dtype, opts, stream);
  if (st != SPKADD_OK) {
    release_all(p);
    clear_trace(p);
    delete p;
    return st;
  }
  *out = p;
  return SPKADD_OK;
}

spkadd_status spkadd_symbolic(spkadd_plan_t p, int32_t* colptr_c, int64_t* nnz_c, hipStream_t stream) {
  g_last_error.clear();
  (void)hipGetLastError();  // a stale status of the caller's earlier HIP calls
  if (!p || !colptr_c || !nnz_c) return set_error(SPKADD_ERR_INVALID, "NULL argument");
  if (p->failed) return set_error(SPKADD_ERR_HIP, "plan failed earlier");
  p->last_stream = stream;
  KArgs a = base_args(p);
  a.alpha_q = p->alpha_sym_q;
  bool wave_done = false;
  if (p->pending) {
    // the wave bins first, from the device's bin lists; then the plan's wait
    if (stream != p->plan_stream && p->ev_sum && hipStreamWaitEvent(stream, p->ev_sum, 0) != hipSuccess) {
      (void)hipGetLastError();
      p->failed = true;
      return set_error(SPKADD_ERR_HIP, "stream wait on the plan failed");
    }
    KArgs fa = a;
    WaveBinTable ft{};
    unsigned fb = 0;
    if (wave_sym_fused_setup(p, fa, ft, fb)) {
      TraceScope t(p, "sym_wave", stream);
      hipError_t e = launch_wave_sym_fused(fa, ft, p->d_list, p->d_binoff, fb, stream);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        p->failed = true;
        return set_error(SPKADD_ERR_HIP, "symbolic launch (sym_wave): %s", hipGetErrorString(e));
      }
      wave_done = true;
    }
    spkadd_status st = plan_finish(p, stream);
    if (st) {
      p->failed = true;
      return st;
    }
    a = base_args(p);  // (the window arrays exist now)
    a.alpha_q = p->alpha_sym_q;
  }
  for (int b = BIN_W1; b < NBINS; ++b) {
    const int cnt = b == BIN_WIN ? p->n_windows : p->bin_count[b];
    if (cnt == 0 || (wave_done && is_wave(b))) continue;
    TraceScope t(p, hash_kernel_name(b, false), stream);
    hipError_t e = launch_bin(p, b, false, a, stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p->failed = true;
      return set_error(SPKADD_ERR_HIP, "symbolic launch (%s): %s", hash_kernel_name(b, false), hipGetErrorString(e));
    }
  }
  if (p->n_windows > 0) {
    TraceScope t(p, "win_colsum", stream);
    launch_win_colsum(p->n_wcols, p->d_list + p->binoff[BIN_WIN], p->d_wfirst, p->d_win_cnt, p->d_colcnt,
                      p->d_win_off, stream);
  }
  {
    TraceScope t(p, "scan", stream);
    launch_scan(p->d_colcnt, p->n, colptr_c, &p->d_sum->total, &p->d_sum->err, p->d_scan_tmp, stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    p->failed = true;
    return set_error(SPKADD_ERR_HIP, "symbolic kernels: %s", hipGetErrorString(e));
  }
  spkadd_status st = sync_summary(p, stream);
  if (st) return st;
  if ((st = check_device_err(p))) return st;
  const long long total = p->h_sum->total;
  if (total > INT_MAX) return set_error(SPKADD_ERR_OVERFLOW, "nnz(B) = %lld exceeds INT32_MAX", total);
  p->colptr_c = colptr_c;
  p->nnz_c = total;
  p->sym_done = true;
  *nnz_c = total;
  return SPKADD_OK;
}

spkadd_status spkadd_numeric(spkadd_plan_t p, const void* const* values, int32_t* rowidx_c, void* values_c,
                             hipStream_t stream) {
  g_last_error.clear();
  (void)hipGetLastError();  // a stale status of the caller's earlier HIP calls
  if (!p) return set_error(SPKADD_ERR_INVALID, "plan is NULL");
  if (p->failed) return set_error(SPKADD_ERR_HIP, "plan failed earlier");
  if (!p->sym_done) return set_error(SPKADD_ERR_STATE, "spkadd_symbolic has not run on this plan");
  if (!values) return set_error(SPKADD_ERR_INVALID, "values is NULL");
  if (p->nnz_c > 0 && (!rowidx_c || !values_c)) return set_error(SPKADD_ERR_INVALID, "output arrays are NULL");
  p->last_stream = stream;
  for (int i = 0; i < p->k; ++i)
    if (!values[i] && p->h_sum->nnz_in > 0) return set_error(SPKADD_ERR_INVALID, "values[%d] is NULL", i);
  {
    TraceScope t(p, "put_ptrs_num", stream, true);
    launch_put_ptrs((const void* const*)values, p->k, p->d_va, nullptr, nullptr, stream);
  }
  KArgs a = base_args(p);
  a.alpha_q = p->alpha_num_q;
  const bool ordered = (p->opts.flags & SPKADD_FLAG_ORDERED) != 0;
  a.unsorted = (p->opts.flags & SPKADD_FLAG_UNSORTED_OUT) && !ordered ? 1 : 0;
  a.colptr_c = p->colptr_c;
  a.out_r = rowidx_c;
  a.out_v = values_c;
  if (p->unsorted_in && p->n_windows > 0) {
    TraceScope t(p, "uwin_gather", stream, true);
    launch_uwin_gather(p->u_total, p->d_ubsrc, (const void* const*)p->d_va, p->d_ubvals,
                       p->dtype == SPKADD_F64, stream);
  }
  for (int b = BIN_W1; b < NBINS; ++b) {
    const int cnt = b == BIN_WIN ? p->n_windows : p->bin_count[b];
    if (cnt == 0) continue;
    TraceScope t(p, hash_kernel_name(b, true), stream, true);
    hipError_t e = launch_bin(p, b, true, a, stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p->failed = true;
      return set_error(SPKADD_ERR_HIP, "numeric launch (%s): %s", hash_kernel_name(b, true), hipGetErrorString(e));
    }
  }
  if (ordered && p->nnz_c > 0) {
    // the rows are in place; every value summed again in input order: wave-bin columns
    // (at most 1024 output entries), then workgroup-bin columns and row windows (at
    // most window_cap)
    const bool f64 = p->dtype == SPKADD_F64;
    const int* wl = p->d_list + p->binoff[BIN_W1];
    const int nw = p->binoff[BIN_G1] - p->binoff[BIN_W1];
    const int* gl = p->d_list + p->binoff[BIN_G1];
    const int ng = p->binoff[BIN_WIN] - p->binoff[BIN_G1];
    TraceScope t(p, "num_ordered", stream, true);
    hipError_t e = launch_ordered(a, wl, nw, 0, kOrderedWaveCap, f64, p->n_cu, stream);
    if (e == hipSuccess) e = launch_ordered(a, gl, ng, p->n_windows, p->pp.cap_in, f64, p->n_cu, stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p->failed = true;
      return set_error(SPKADD_ERR_HIP, "numeric launch (ordered values): %s", hipGetErrorString(e));
    }
  }
  return SPKADD_OK;
}

spkadd_status spkadd_free(spkadd_plan_t p) {
  if (!p) return SPKADD_OK;
  release_all(p);
  clear_trace(p);
  delete p;
  return SPKADD_OK;
}

spkadd_status spkadd_get_stats(spkadd_plan_t p, spkadd_stats* out) {
  if (!p || !out) return set_error(SPKADD_ERR_INVALID, "NULL argument");
  if (p->pending) {
    const spkadd_status st = plan_finish(p, p->last_stream);
    if (st) {
      p->failed = true;
      return st;
    }
  }
  spkadd_stats s{};
  s.nnz_in = (int64_t)p->h_sum->nnz_in;
  s.nnz_out = p->sym_done ? p->nnz_c : -1;
  s.n_empty_cols = p->bin_count[BIN_EMPTY];
  for (int b = BIN_W1; b <= BIN_W16; ++b) s.n_wave_cols += p->bin_count[b];
  s.n_wg_cols = p->bin_count[BIN_G1] + p->bin_count[BIN_G2];
  s.n_window_cols = p->n_wcols;
  s.n_windows = p->n_windows;
  s.window_levels = p->levels;
  s.window_cap = p->pp.cap_in;
  s.wave_max = p->pp.force_bin == 0 ? 1024 : p->pp.wave_max;
  // device error flags raised by numeric passes since the last wait
  if (sync_summary(p, p->last_stream) != SPKADD_OK) (void)hipGetLastError();
  *out = s;
  return check_device_err(p);
}

int32_t spkadd_trace_count(spkadd_plan_t p) { return p ? (int32_t)p->trace.size() : 0; }

spkadd_status spkadd_trace_get(spkadd_plan_t p, int32_t idx, char* name, int32_t name_cap, float* ms) {
  if (!p || idx < 0 || idx >= (int32_t)p->trace.size()) return set_error(SPKADD_ERR_INVALID, "bad trace index");
  const TraceRec& r = p->trace[(size_t)idx];
  if (name && name_cap > 0) {
    strncpy(name, r.name, (size_t)name_cap - 1);
    name[name_cap - 1] = 0;
  }
  if (ms) {
    HIP_TRY(hipEventSynchronize(r.b));
    HIP_TRY(hipEventElapsedTime(ms, r.a, r.b));
  }
  return SPKADD_OK;
}

spkadd_status spkadd_trace_reset(spkadd_plan_t p) {
  if (!p) return set_error(SPKADD_ERR_INVALID, "plan is NULL");
  clear_trace(p);
  return SPKADD_OK;
}

}  // extern "C"

namespace spk {

spkadd_status sum_in_region(void* region, size_t region_bytes, int32_t m, int32_t n, int32_t k,
                            const int32_t* const* colptr, const int32_t* const* rowidx, const void* const* values,
                            spkadd_dtype dtype, const spkadd_opts* opts, int32_t* colptr_c, int32_t* rowidx_c,
                            void* values_c, int64_t cap_c, int64_t* nnz_c, hipStream_t stream) {
  g_last_error.clear();
  (void)hipGetLastError();  // a stale status of the caller's earlier HIP calls
  if (!nnz_c || !colptr_c || !values) return set_error(SPKADD_ERR_INVALID, "NULL argument");
  *nnz_c = -1;
  if (cap_c < 0) return set_error(SPKADD_ERR_INVALID, "cap_c must be >= 0");
  spkadd_opts o;
  spkadd_opts_default(&o);
  if (opts) o = *opts;
  o.flags &= ~(SPKADD_FLAG_TRACE | SPKADD_FLAG_TRACE_NUMERIC);  // (traces take events)
  spkadd_plan_s p;
  p.region_mode = true;
  p.region = (char*)region;
  p.region_bytes = region_bytes;
  spkadd_status st = plan_build(&p, m, n, k, colptr, rowidx, dtype, &o, stream);
  int64_t nnz = -1;
  if (st == SPKADD_OK) st = spkadd_symbolic(&p, colptr_c, &nnz, stream);
  if (st == SPKADD_OK) {
    *nnz_c = nnz;
    if (nnz > cap_c)
      st = set_error(SPKADD_ERR_INVALID, "nnz(B) = %lld exceeds cap_c = %lld (colptr_c and *nnz_c are written)",
                     (long long)nnz, (long long)cap_c);
  }
  if (st == SPKADD_OK) st = spkadd_numeric(&p, values, rowidx_c, values_c, stream);
  release_all(&p);
  return st;
}

}  // namespace spk
