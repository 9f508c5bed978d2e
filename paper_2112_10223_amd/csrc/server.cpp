// The serving loop of include/spkadd_server.h: a server thread admits queued
// requests by HBM budget into batched runs rotating over several streams; a second
// thread runs the requests that are too large for a batch through the one-request
// path.  Tickets complete with timestamps on one steady clock.
#include "spkadd_server.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace spk;

namespace {

spkadd_status sfail(spkadd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return report_error(st, buf);
}

enum class TState { Pending, Running, Large, Done };

struct Ticket {
  uint64_t id = 0;
  int m = 0, n = 0, k = 0;
  long long cap = 0;
  std::vector<const void*> cp, ri, va;
  size_t bytes = 0;       // output memory
  char* out = nullptr;    // one block: colptr(B), rows, values
  TState state = TState::Pending;
  spkadd_result res{};
};

struct InFlight {
  spkadd_batch_t batch;
  std::vector<uint64_t> ids;
};

struct Lane {  // one stream and its two batch objects
  hipStream_t stream = nullptr;
  spkadd_batch_t batch[2] = {nullptr, nullptr};
  std::deque<InFlight> inflight;
  int next = 0;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t size_class(size_t bytes) {
  size_t c = 64 * 1024;
  while (c < bytes) c <<= 1;
  return c;
}

}  // namespace

struct spkadd_server_s {
  spkadd_server_config cfg{};
  spkadd_opts opts{};
  int device = 0;
  int vbytes = 4;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending, large;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_id = 1;
  uint64_t in_use = 0;
  bool stop = false;
  std::vector<Lane> lanes;
  std::vector<hipStream_t> large_streams;  // one per one-request lane
  hipStream_t free_stream = nullptr;
  // released output blocks by size class (power of two, >= 64 KiB), reused by later
  // requests; held blocks and pooled ones together stay within the budget
  std::unordered_map<size_t, std::vector<char*>> pool;
  uint64_t pooled = 0;
  long long runs = 0, batched = 0, large_count = 0, allocations = 0;
  std::thread loop;
  std::vector<std::thread> large_loops;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// status: SPKADD_REQ_OK / SPKADD_REQ_CAPACITY, or an spkadd_status error (> 0 and not
// an outcome) passed as -error.
void complete(spkadd_server_s* s, Ticket& t, int status, long long nnz, int path) {
  t.res.status = status >= 0 ? status : SPKADD_REQ_ERROR;
  t.res.error = status >= 0 ? SPKADD_OK : -status;
  t.res.path = path;
  t.res.nnz = nnz;
  t.res.t_done = s->now();
  t.state = TState::Done;
}

// Retires the finished runs at the front of a lane (caller holds the lock).
bool retire(spkadd_server_s* s, Lane& ln) {
  bool any = false;
  while (!ln.inflight.empty()) {
    InFlight& f = ln.inflight.front();
    if (!spkadd_batch_ready(f.batch)) break;  // runs of a lane finish in order
    std::vector<int64_t> nnz(f.ids.size());
    std::vector<int32_t> st(f.ids.size());
    const spkadd_status rs = spkadd_batch_results(f.batch, nnz.data(), st.data());
    for (size_t i = 0; i < f.ids.size(); ++i) {
      Ticket& t = s->tickets[f.ids[i]];
      if (rs != SPKADD_OK) {
        complete(s, t, -(int)rs, -1, 0);
      } else if (st[i] == SPKADD_REQ_TOO_LARGE) {
        t.state = TState::Large;
        s->large.push_back(t.id);
      } else {
        complete(s, t, st[i], nnz[i], 0);
      }
    }
    ln.inflight.pop_front();
    any = true;
  }
  return any;
}

// Frees pooled blocks until `bytes` more fit the budget beside the held and pooled
// ones (caller holds the lock).  Pooled blocks are idle: their tickets completed.
void evict(spkadd_server_s* s, size_t bytes) {
  for (auto it = s->pool.begin(); it != s->pool.end() && s->in_use + s->pooled + bytes > s->cfg.hbm_budget; ++it) {
    while (!it->second.empty() && s->in_use + s->pooled + bytes > s->cfg.hbm_budget) {
      (void)hipFreeAsync(it->second.back(), s->free_stream);
      it->second.pop_back();
      s->pooled -= it->first;
    }
  }
}

// Forms one batched run on a lane with a free batch object (caller holds the lock).
bool admit(spkadd_server_s* s, Lane& ln) {
  if (s->pending.empty() || (int)ln.inflight.size() >= s->cfg.depth) return false;
  std::vector<uint64_t> ids;
  std::vector<spkadd_request> reqs;
  long long cols = 0, inputs = 0;
  while (!s->pending.empty() && (int)ids.size() < s->cfg.max_batch) {
    Ticket& t = s->tickets[s->pending.front()];
    if (cols + t.n > s->cfg.max_columns || inputs + t.k > s->cfg.max_inputs) break;
    if (s->in_use + t.bytes > s->cfg.hbm_budget) break;
    auto& fl = s->pool[t.bytes];
    if (!fl.empty()) {
      t.out = fl.back();
      fl.pop_back();
      s->pooled -= t.bytes;
    } else {
      evict(s, t.bytes);
      if (hipMallocAsync((void**)&t.out, t.bytes, ln.stream) != hipSuccess) {
        (void)hipGetLastError();
        t.out = nullptr;
        break;
      }
      ++s->allocations;
    }
    s->in_use += t.bytes;
    cols += t.n;
    inputs += t.k;
    t.res.colptr_c = (int32_t*)t.out;
    t.res.rowidx_c = (int32_t*)(t.out + align_up((size_t)(t.n + 1) * 4, 256));
    t.res.values_c = t.out + align_up((size_t)(t.n + 1) * 4, 256) + align_up((size_t)t.cap * 4 + 4, 256);
    spkadd_request q{};
    q.m = t.m;
    q.n = t.n;
    q.k = t.k;
    q.colptr = (const int32_t* const*)t.cp.data();
    q.rowidx = (const int32_t* const*)t.ri.data();
    q.values = t.va.data();
    q.colptr_c = t.res.colptr_c;
    q.rowidx_c = t.res.rowidx_c;
    q.values_c = t.res.values_c;
    q.cap_c = t.cap;
    reqs.push_back(q);
    ids.push_back(t.id);
    t.state = TState::Running;
    t.res.t_start = s->now();
    s->pending.pop_front();
  }
  if (ids.empty()) return false;
  // the lane's batch object that no run in flight uses (depth <= 2, two objects)
  int slot = ln.next;
  for (const InFlight& f : ln.inflight)
    if (f.batch == ln.batch[slot]) slot ^= 1;
  spkadd_batch_t b = ln.batch[slot];
  const spkadd_status st = spkadd_batch_run(b, reqs.data(), (int32_t)reqs.size(), 1, ln.stream);
  if (st == SPKADD_OK) ln.next = slot ^ 1;  // a failed run leaves the object free for the next
  if (st != SPKADD_OK) {
    for (uint64_t id : ids) complete(s, s->tickets[id], -(int)st, -1, 0);
    s->cv_done.notify_all();
    return true;
  }
  ln.inflight.push_back(InFlight{b, ids});
  ++s->runs;
  s->batched += (long long)ids.size();
  return true;
}

// How long the server thread keeps polling after its last work before it sleeps on
// the condition variable (waking from it costs tens of microseconds), and how long a
// waiting client polls its ticket before it sleeps.
constexpr auto kIdleSpin = std::chrono::microseconds(500);
constexpr auto kWaitSpin = std::chrono::microseconds(2000);

void server_loop(spkadd_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  auto last_work = std::chrono::steady_clock::now();
  for (;;) {
    bool progress = false;
    for (Lane& ln : s->lanes) progress |= retire(s, ln);
    if (progress) s->cv_done.notify_all();
    if (!s->large.empty()) s->cv_work.notify_all();
    for (Lane& ln : s->lanes) progress |= admit(s, ln);
    bool running = !s->large.empty();
    for (Lane& ln : s->lanes) running |= !ln.inflight.empty();
    if (s->stop && !running) {  // requests never admitted are cancelled
      for (uint64_t id : s->pending) complete(s, s->tickets[id], -(int)SPKADD_ERR_STATE, -1, 0);
      s->pending.clear();
      s->cv_done.notify_all();
      break;
    }
    if (progress) {
      last_work = std::chrono::steady_clock::now();
      continue;
    }
    if (running || std::chrono::steady_clock::now() - last_work < kIdleSpin) {
      // runs in flight, or idle only briefly: poll every few microseconds (a timed
      // wait on the condition variable wakes up far later than asked)
      lk.unlock();
      const auto t1 = std::chrono::steady_clock::now();
      while (std::chrono::steady_clock::now() - t1 < std::chrono::microseconds(5)) std::this_thread::yield();
      lk.lock();
    } else {
      s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

// Requests too large for a batch: plan / symbolic / numeric on a stream of their own
// (one-request lane `lane`; the lanes take requests from one queue, in order).
void large_loop(spkadd_server_s* s, int lane) {
  hipStream_t stream = s->large_streams[(size_t)lane];
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->large.empty()) {
      bool busy = false;
      for (Lane& ln : s->lanes) busy |= !ln.inflight.empty();
      if (s->stop && !busy) break;
      s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    const uint64_t id = s->large.front();
    s->large.pop_front();
    ++s->large_count;
    Ticket& t = s->tickets[id];
    const int m = t.m, n = t.n, k = t.k;
    const long long cap = t.cap;
    auto cp = t.cp;
    auto ri = t.ri;
    auto va = t.va;
    spkadd_result res = t.res;
    lk.unlock();
    spkadd_plan_t p = nullptr;
    long long nnz = -1;
    int outcome = SPKADD_REQ_OK;
    spkadd_status st = spkadd_plan(&p, m, n, k, (const int32_t* const*)cp.data(), (const int32_t* const*)ri.data(),
                                   s->cfg.dtype, &s->opts, stream);
    if (st == SPKADD_OK) {
      int64_t z = 0;
      st = spkadd_symbolic(p, res.colptr_c, &z, stream);
      nnz = z;
      if (st == SPKADD_OK && z > cap) outcome = SPKADD_REQ_CAPACITY;
      if (st == SPKADD_OK && outcome == SPKADD_REQ_OK)
        st = spkadd_numeric(p, va.data(), res.rowidx_c, res.values_c, stream);
      if (st == SPKADD_OK && hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        st = SPKADD_ERR_HIP;
      }
    }
    spkadd_free(p);
    const int status = st != SPKADD_OK ? -(int)st : outcome;
    lk.lock();
    complete(s, s->tickets[id], status, nnz, 1);
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

double spkadd_server_now(spkadd_server_t s) { return s ? s->now() : 0.0; }

spkadd_status spkadd_server_create(spkadd_server_t* out, const spkadd_server_config* cfg) {
  if (!out || !cfg) return sfail(SPKADD_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (cfg->dtype != SPKADD_F32 && cfg->dtype != SPKADD_F64) return sfail(SPKADD_ERR_INVALID, "bad dtype");
  if (cfg->n_streams < 1 || cfg->n_streams > 8) return sfail(SPKADD_ERR_INVALID, "n_streams must be 1..8");
  if (cfg->max_batch < 0 || cfg->max_batch > 4096) return sfail(SPKADD_ERR_INVALID, "max_batch must be 0..4096");
  if (cfg->depth < 1 || cfg->depth > 2) return sfail(SPKADD_ERR_INVALID, "depth must be 1 or 2");
  if (cfg->large_streams < 0 || cfg->large_streams > 8) return sfail(SPKADD_ERR_INVALID, "large_streams must be 0..8");
  if (cfg->max_columns < 1 || cfg->max_inputs < 1 || cfg->hbm_budget == 0)
    return sfail(SPKADD_ERR_INVALID, "max_columns, max_inputs and hbm_budget must be positive");
  auto* s = new (std::nothrow) spkadd_server_s();
  if (!s) return sfail(SPKADD_ERR_OOM, "host allocation failed");
  s->cfg = *cfg;
  spkadd_opts_default(&s->opts);
  if (cfg->opts) s->opts = *cfg->opts;
  s->cfg.opts = nullptr;
  if (s->cfg.large_streams == 0) s->cfg.large_streams = 2;
  if (s->cfg.max_batch == 0)  // the tuned run size, else 8
    s->cfg.max_batch = s->opts.batch_run_size > 0 && s->opts.batch_run_size <= 4096 ? s->opts.batch_run_size : 8;
  s->vbytes = cfg->dtype == SPKADD_F64 ? 8 : 4;
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return sfail(SPKADD_ERR_HIP, "no HIP device");
  }
  auto cleanup = [&](spkadd_status st, const char* what) {
    for (Lane& ln : s->lanes) {
      for (auto& b : ln.batch) spkadd_batch_destroy(b);
      if (ln.stream) (void)hipStreamDestroy(ln.stream);
    }
    for (hipStream_t ls : s->large_streams)
      if (ls) (void)hipStreamDestroy(ls);
    if (s->free_stream) (void)hipStreamDestroy(s->free_stream);
    delete s;
    return sfail(st, "%s", what);
  };
  s->lanes.resize((size_t)cfg->n_streams);
  for (Lane& ln : s->lanes) {
    if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess) return cleanup(SPKADD_ERR_HIP, "stream");
    for (auto& b : ln.batch) {
      const spkadd_status st =
          spkadd_batch_create(&b, cfg->dtype, s->cfg.max_batch, cfg->max_columns, cfg->max_inputs, &s->opts);
      if (st != SPKADD_OK) return cleanup(st, "batch creation failed");
    }
  }
  s->large_streams.assign((size_t)s->cfg.large_streams, nullptr);
  for (hipStream_t& ls : s->large_streams)
    if (hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) != hipSuccess) return cleanup(SPKADD_ERR_HIP, "stream");
  if (hipStreamCreateWithFlags(&s->free_stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(SPKADD_ERR_HIP, "stream");
  s->loop = std::thread(server_loop, s);
  for (int l = 0; l < s->cfg.large_streams; ++l) s->large_loops.emplace_back(large_loop, s, l);
  *out = s;
  return SPKADD_OK;
}

spkadd_status spkadd_server_submit(spkadd_server_t s, const spkadd_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return sfail(SPKADD_ERR_INVALID, "NULL argument");
  if (req->k < 1 || req->k > 64) return sfail(SPKADD_ERR_INVALID, "k = %d (1..64)", req->k);
  if (req->m < 0 || req->n < 0 || req->m == INT32_MAX || req->n == INT32_MAX || req->cap_c < 0)
    return sfail(SPKADD_ERR_INVALID, "bad shape or capacity");
  if (!req->colptr || !req->rowidx || !req->values) return sfail(SPKADD_ERR_INVALID, "NULL pointer arrays");
  if (req->n > s->cfg.max_columns || req->k > s->cfg.max_inputs)
    return sfail(SPKADD_ERR_INVALID, "request larger than one batched run");
  Ticket t;
  t.m = req->m;
  t.n = req->n;
  t.k = req->k;
  t.cap = req->cap_c;
  for (int i = 0; i < req->k; ++i) {
    if (!req->colptr[i] || !req->rowidx[i] || !req->values[i])
      return sfail(SPKADD_ERR_INVALID, "input %d has a NULL array", i);
    t.cp.push_back(req->colptr[i]);
    t.ri.push_back(req->rowidx[i]);
    t.va.push_back(req->values[i]);
  }
  t.bytes = size_class(align_up((size_t)(t.n + 1) * 4, 256) + align_up((size_t)t.cap * 4 + 4, 256) +
                       align_up((size_t)t.cap * (size_t)s->vbytes + 8, 256));
  if (t.bytes > s->cfg.hbm_budget) return sfail(SPKADD_ERR_INVALID, "request outputs exceed the budget");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return sfail(SPKADD_ERR_STATE, "server is stopping");
  t.id = s->next_id++;
  t.res.t_submit = s->now();
  const uint64_t id = t.id;
  s->tickets.emplace(id, std::move(t));
  s->pending.push_back(id);
  *ticket = id;
  s->cv_work.notify_all();
  return SPKADD_OK;
}

spkadd_status spkadd_server_wait(spkadd_server_t s, uint64_t ticket, spkadd_result* out, double timeout_s) {
  if (!s) return sfail(SPKADD_ERR_INVALID, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return sfail(SPKADD_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  auto done = [&] { return s->tickets[ticket].state == TState::Done; };
  // poll for a short while first: most tickets complete within it
  const auto t0 = std::chrono::steady_clock::now();
  while (!done() && std::chrono::steady_clock::now() - t0 < kWaitSpin &&
         (timeout_s < 0 || std::chrono::steady_clock::now() - t0 < std::chrono::duration<double>(timeout_s))) {
    lk.unlock();
    std::this_thread::yield();
    lk.lock();
  }
  if (timeout_s < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return sfail(SPKADD_ERR_STATE, "ticket %llu still pending", (unsigned long long)ticket);
  }
  if (out) *out = s->tickets[ticket].res;
  return SPKADD_OK;
}

spkadd_status spkadd_server_release(spkadd_server_t s, uint64_t ticket) {
  if (!s) return sfail(SPKADD_ERR_INVALID, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return sfail(SPKADD_ERR_INVALID, "unknown ticket");
  if (it->second.state != TState::Done) return sfail(SPKADD_ERR_STATE, "ticket not complete");
  if (it->second.out) {
    // kept for reuse: the ticket's work is complete, so the block is idle
    s->pool[it->second.bytes].push_back(it->second.out);
    s->pooled += it->second.bytes;
    s->in_use -= it->second.bytes;
  }
  s->tickets.erase(it);
  s->cv_work.notify_all();
  return SPKADD_OK;
}

spkadd_status spkadd_server_get_info(spkadd_server_t s, spkadd_server_info* out) {
  if (!s || !out) return sfail(SPKADD_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);  // the batch objects are used under this lock only
  *out = spkadd_server_info{};
  out->runs = s->runs;
  out->batched = s->batched;
  out->large = s->large_count;
  out->allocations = s->allocations;
  out->held_bytes = s->in_use;
  out->pooled_bytes = s->pooled;
  for (Lane& ln : s->lanes)
    for (auto& b : ln.batch) {
      spkadd_batch_info bi{};
      if (spkadd_batch_get_info(b, &bi) == SPKADD_OK) {
        out->graphs_captured += bi.graphs_captured;
        out->graph_reuses += bi.graph_reuses;
      }
    }
  return SPKADD_OK;
}

spkadd_status spkadd_server_destroy(spkadd_server_t s) {
  if (!s) return SPKADD_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  s->loop.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_work.notify_all();
  }
  for (std::thread& th : s->large_loops) th.join();
  for (Lane& ln : s->lanes) {
    (void)hipStreamSynchronize(ln.stream);
    for (auto& b : ln.batch) spkadd_batch_destroy(b);
  }
  for (hipStream_t ls : s->large_streams) (void)hipStreamSynchronize(ls);
  for (auto& kv : s->tickets)
    if (kv.second.out) (void)hipFreeAsync(kv.second.out, s->free_stream);
  for (auto& kv : s->pool)
    for (char* p : kv.second) (void)hipFreeAsync(p, s->free_stream);
  (void)hipStreamSynchronize(s->free_stream);
  for (Lane& ln : s->lanes) (void)hipStreamDestroy(ln.stream);
  for (hipStream_t ls : s->large_streams) (void)hipStreamDestroy(ls);
  (void)hipStreamDestroy(s->free_stream);
  delete s;
  return SPKADD_OK;
}

}  // extern "C"
