// Autotuner of include/spkadd_tune.h: coordinate descent over the launch parameters
// measured on the caller's inputs, a process-wide cache keyed by shape class, and its
// JSON file format (written and read here, no external library).
#include "spkadd_tune.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "spkadd_batch.h"

using namespace spk;

namespace {

spkadd_status tfail(spkadd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return report_error(st, buf);
}

int ceil_log2_ll(long long x) {
  int r = 0;
  while (x > 1 && (1LL << r) < x) ++r;
  return x <= 1 ? 0 : r;
}

// The fields the tuner sets.  A one-request entry (key kind 0) sets the first group,
// a batched entry (kind 1) the accumulator choice and the batch group.
struct Tuned {
  int wave_max = 0, accum_mode = 0, wave_merge = 0, window_cap = 0;
  float bitmap_ratio = 0.f, load_factor_sym = 0.f, load_factor_num = 0.f, window_fill = 0.f;
  int batch_fused_cols = 0, batch_wave_max = 0, batch_wg_max = 0, batch_wg_threads = 0, batch_run_size = 0;
  double ms = -1.0;
};

Tuned tuned_of(const spkadd_opts& o, double ms) {
  Tuned t;
  t.wave_max = o.wave_max;
  t.accum_mode = o.accum_mode;
  t.wave_merge = o.wave_merge;
  t.window_cap = o.window_cap;
  t.bitmap_ratio = o.bitmap_ratio;
  t.load_factor_sym = o.load_factor_sym;
  t.load_factor_num = o.load_factor_num;
  t.window_fill = o.window_fill;
  t.batch_fused_cols = o.batch_fused_cols;
  t.batch_wave_max = o.batch_wave_max;
  t.batch_wg_max = o.batch_wg_max;
  t.batch_wg_threads = o.batch_wg_threads;
  t.batch_run_size = o.batch_run_size;
  t.ms = ms;
  return t;
}

void apply(const Tuned& t, int kind, spkadd_opts& o) {
  o.accum_mode = t.accum_mode;
  o.bitmap_ratio = t.bitmap_ratio;
  if (kind == 1) {
    o.batch_fused_cols = t.batch_fused_cols;
    o.batch_wave_max = t.batch_wave_max;
    o.batch_wg_max = t.batch_wg_max;
    o.batch_wg_threads = t.batch_wg_threads;
    o.batch_run_size = t.batch_run_size;
    return;
  }
  o.wave_max = t.wave_max;
  o.wave_merge = t.wave_merge;
  o.window_cap = t.window_cap;
  o.load_factor_sym = t.load_factor_sym;
  o.load_factor_num = t.load_factor_num;
  o.window_fill = t.window_fill;
}

using KeyTuple = std::tuple<std::string, int, int, int, int, int, int, int>;

KeyTuple key_tuple(const spkadd_tune_key& k) {
  char arch[sizeof(k.arch) + 1];
  memcpy(arch, k.arch, sizeof(k.arch));
  arch[sizeof(k.arch)] = 0;
  return KeyTuple(std::string(arch), k.cus, k.dtype, k.m_log2, k.n_log2, k.k_log2, k.u_log2, k.kind);
}

struct Cache {
  std::mutex mu;
  std::map<KeyTuple, Tuned> entries;
};

// Never destroyed, like the library's other process-wide caches: no static
// destructor of the library runs at process exit.
Cache& cache() {
  static Cache* c = new Cache();
  return *c;
}

bool valid_key(const spkadd_tune_key* k) {
  return k && memchr(k->arch, 0, sizeof(k->arch)) != nullptr && k->cus >= 0 && (k->dtype == 0 || k->dtype == 1) &&
         k->m_log2 >= 0 && k->m_log2 <= 31 && k->n_log2 >= 0 && k->n_log2 <= 31 && k->k_log2 >= 0 &&
         k->k_log2 <= 31 && k->u_log2 >= 0 && k->u_log2 <= 40 && (k->kind == 0 || k->kind == 1);
}

// ---- JSON: the cache's own format, a list of flat objects ----

void put_str(std::string& s, const std::string& v) {
  s += '"';
  for (char c : v) {
    if (c == '"' || c == '\\') s += '\\';
    if ((unsigned char)c < 0x20) continue;
    s += c;
  }
  s += '"';
}

struct JVal {
  enum Kind { Null, Num, Str, Arr, Obj, Bool } kind = Null;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* name) const {
    for (auto& kv : obj)
      if (kv.first == name) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  int depth = 0;
  void ws() {
    while (p < end && isspace((unsigned char)*p)) ++p;
  }
  bool lit(const char* w) {
    const size_t n = strlen(w);
    if ((size_t)(end - p) < n || strncmp(p, w, n) != 0) return false;
    p += n;
    return true;
  }
  bool string(std::string& out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      if (*p == '\\') {
        if (++p >= end) return false;
        const char c = *p;
        if (c == 'n') out += '\n';
        else if (c == 't') out += '\t';
        else if (c == '"' || c == '\\' || c == '/') out += c;
        else return false;  // no other escapes are written
        ++p;
      } else {
        out += *p++;
      }
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool value(JVal& v) {
    if (++depth > 8) return false;
    ws();
    if (p >= end) return false;
    bool ok = true;
    if (*p == '{') {
      v.kind = JVal::Obj;
      ++p;
      ws();
      if (p < end && *p == '}') {
        ++p;
      } else {
        for (;;) {
          ws();
          std::string name;
          if (!string(name)) return false;
          ws();
          if (p >= end || *p != ':') return false;
          ++p;
          JVal x;
          if (!value(x)) return false;
          v.obj.emplace_back(std::move(name), std::move(x));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == '}') {
            ++p;
            break;
          }
          return false;
        }
      }
    } else if (*p == '[') {
      v.kind = JVal::Arr;
      ++p;
      ws();
      if (p < end && *p == ']') {
        ++p;
      } else {
        for (;;) {
          JVal x;
          if (!value(x)) return false;
          v.arr.push_back(std::move(x));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == ']') {
            ++p;
            break;
          }
          return false;
        }
      }
    } else if (*p == '"') {
      v.kind = JVal::Str;
      ok = string(v.str);
    } else if (lit("null")) {
      v.kind = JVal::Null;
    } else if (lit("true")) {
      v.kind = JVal::Bool;
      v.num = 1;
    } else if (lit("false")) {
      v.kind = JVal::Bool;
    } else {
      char* q = nullptr;
      std::string tok;
      while (p < end && (isdigit((unsigned char)*p) || *p == '-' || *p == '+' || *p == '.' || *p == 'e' || *p == 'E'))
        tok += *p++;
      if (tok.empty()) return false;
      v.kind = JVal::Num;
      v.num = strtod(tok.c_str(), &q);
      ok = q && *q == 0 && std::isfinite(v.num);
    }
    --depth;
    return ok;
  }
};

bool num_field(const JVal& o, const char* name, double lo, double hi, double* out) {
  const JVal* v = o.get(name);
  if (!v || v->kind != JVal::Num || !(v->num >= lo && v->num <= hi)) return false;
  *out = v->num;
  return true;
}

bool int_field(const JVal& o, const char* name, int lo, int hi, int* out) {
  double d = 0;
  if (!num_field(o, name, lo, hi, &d) || d != std::floor(d)) return false;
  *out = (int)d;
  return true;
}

// ---- measurement ----

struct Trial {
  spkadd_opts o;
  double ms = -1;
  spkadd_status st = SPKADD_OK;
  bool same = false;
};

struct Runner {
  int m, n, k;
  const int32_t* const* cp;
  const int32_t* const* ri;
  const void* const* va;
  spkadd_dtype dtype;
  int reps;
  hipStream_t stream;
  int32_t* d_colptr = nullptr;
  int32_t* d_rows = nullptr;
  void* d_vals = nullptr;
  std::vector<int32_t> ref, got;
  bool have_ref = false;
  long long nnz_ref = -1;

  spkadd_status once(const spkadd_opts& o, long long* nnz) {
    spkadd_plan_t p = nullptr;
    spkadd_status st = spkadd_plan(&p, m, n, k, cp, ri, dtype, &o, stream);
    int64_t z = 0;
    if (st == SPKADD_OK) st = spkadd_symbolic(p, d_colptr, &z, stream);
    if (st == SPKADD_OK) st = spkadd_numeric(p, va, d_rows, d_vals, stream);
    if (st == SPKADD_OK && hipStreamSynchronize(stream) != hipSuccess) {
      (void)hipGetLastError();
      st = tfail(SPKADD_ERR_HIP, "stream synchronisation failed");
    }
    spkadd_free(p);
    *nnz = z;
    return st;
  }

  void measure(Trial& t) {
    long long z = -1;
    t.st = once(t.o, &z);  // untimed: first use of the setting
    if (t.st != SPKADD_OK) return;
    if (hipMemcpy(got.data(), d_colptr, got.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      t.st = SPKADD_ERR_HIP;
      return;
    }
    if (!have_ref) {
      ref = got;
      nnz_ref = z;
      have_ref = true;
    }
    t.same = z == nnz_ref && got == ref;
    std::vector<double> ts;
    for (int r = 0; r < reps && t.st == SPKADD_OK; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      t.st = once(t.o, &z);
      ts.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    if (t.st != SPKADD_OK) return;
    std::sort(ts.begin(), ts.end());
    t.ms = ts[ts.size() / 2];
  }
};

// A trial of the batched path: every request of the sample in runs of `run` requests
// through two batch objects that alternate, then the requests reported too large
// through the one-request path (as the serving loop does).
struct BatchRunner {
  const spkadd_request* reqs;
  int nreq;
  spkadd_dtype dtype;
  int reps;
  hipStream_t stream;
  std::vector<long long> ref;
  bool have_ref = false;

  static int run_of(const spkadd_opts& o, int nreq) {
    const int r = o.batch_run_size > 0 ? o.batch_run_size : 8;
    return r < nreq ? r : nreq;
  }

  spkadd_status pass(const spkadd_opts& o, spkadd_batch_t* bt, int R, std::vector<long long>& nnz) {
    nnz.assign((size_t)nreq, -1);
    std::vector<int> large;
    std::vector<int64_t> gz((size_t)R);
    std::vector<int32_t> gs((size_t)R);
    int pending[2] = {-1, -1};
    auto collect = [&](int slot) -> spkadd_status {
      const int g = pending[slot];
      if (g < 0) return SPKADD_OK;
      const spkadd_status st = spkadd_batch_results(bt[slot], gz.data(), gs.data());
      if (st != SPKADD_OK) return st;
      for (int r = g * R, t = 0; r < nreq && t < R; ++r, ++t) {
        if (gs[(size_t)t] == SPKADD_REQ_TOO_LARGE) large.push_back(r);
        else nnz[(size_t)r] = gz[(size_t)t];
      }
      pending[slot] = -1;
      return SPKADD_OK;
    };
    const int groups = (nreq + R - 1) / R;
    for (int g = 0; g < groups; ++g) {
      const int slot = g & 1;
      spkadd_status st = collect(slot);
      if (st != SPKADD_OK) return st;
      const int cnt = nreq - g * R < R ? nreq - g * R : R;
      st = spkadd_batch_run(bt[slot], reqs + (size_t)g * R, cnt, 1, stream);
      if (st != SPKADD_OK) return st;
      pending[slot] = g;
    }
    for (int slot = 0; slot < 2; ++slot) {
      const spkadd_status st = collect(groups % 2 == 0 ? slot : 1 - slot);
      if (st != SPKADD_OK) return st;
    }
    for (int r : large) {
      const spkadd_request& q = reqs[r];
      spkadd_plan_t p = nullptr;
      spkadd_status st = spkadd_plan(&p, q.m, q.n, q.k, q.colptr, q.rowidx, dtype, &o, stream);
      int64_t z = -1;
      if (st == SPKADD_OK) st = spkadd_symbolic(p, q.colptr_c, &z, stream);
      if (st == SPKADD_OK && z <= q.cap_c) st = spkadd_numeric(p, q.values, q.rowidx_c, q.values_c, stream);
      spkadd_free(p);
      if (st != SPKADD_OK) return st;
      nnz[(size_t)r] = z;
    }
    if (hipStreamSynchronize(stream) != hipSuccess) {
      (void)hipGetLastError();
      return tfail(SPKADD_ERR_HIP, "stream synchronisation failed");
    }
    return SPKADD_OK;
  }

  void measure(Trial& t) {
    const int R = run_of(t.o, nreq);
    long long cols = 0, inputs = 0;
    for (int g = 0; g * R < nreq; ++g) {
      long long c = 0, i = 0;
      for (int r = g * R; r < nreq && r < (g + 1) * R; ++r) {
        c += reqs[r].n;
        i += reqs[r].k;
      }
      cols = c > cols ? c : cols;
      inputs = i > inputs ? i : inputs;
    }
    spkadd_batch_t bt[2] = {nullptr, nullptr};
    for (auto& b : bt) {
      t.st = spkadd_batch_create(&b, dtype, R, cols > 0 ? cols : 1, inputs > 0 ? inputs : 1, &t.o);
      if (t.st != SPKADD_OK) break;
    }
    std::vector<long long> nnz;
    if (t.st == SPKADD_OK) t.st = pass(t.o, bt, R, nnz);  // untimed: graphs captured
    if (t.st == SPKADD_OK) {
      if (!have_ref) {
        ref = nnz;
        have_ref = true;
      }
      t.same = nnz == ref;
      std::vector<double> ts;
      for (int r = 0; r < reps && t.st == SPKADD_OK; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        t.st = pass(t.o, bt, R, nnz);
        ts.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        t.same = t.same && nnz == ref;
      }
      if (t.st == SPKADD_OK) {
        std::sort(ts.begin(), ts.end());
        t.ms = ts[ts.size() / 2];
      }
    }
    for (auto& b : bt) spkadd_batch_destroy(b);
  }
};

}  // namespace

extern "C" {

spkadd_status spkadd_tune_key_for(int32_t m, int32_t n, int32_t k, int64_t nnz_in, spkadd_dtype dtype,
                                  spkadd_tune_key* out) {
  if (!out) return tfail(SPKADD_ERR_INVALID, "out is NULL");
  if (m < 0 || n < 0 || k < 1 || nnz_in < 0 || (dtype != SPKADD_F32 && dtype != SPKADD_F64))
    return tfail(SPKADD_ERR_INVALID, "bad shape, count or dtype");
  memset(out, 0, sizeof(*out));
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return tfail(SPKADD_ERR_HIP, "no HIP device");
  }
  snprintf(out->arch, sizeof(out->arch), "%s", prop.gcnArchName);
  out->cus = prop.multiProcessorCount;
  out->dtype = (int32_t)dtype;
  out->m_log2 = ceil_log2_ll(m);
  out->n_log2 = ceil_log2_ll(n);
  out->k_log2 = ceil_log2_ll(k);
  out->u_log2 = n > 0 ? ceil_log2_ll((nnz_in + n - 1) / n) : 0;
  return SPKADD_OK;
}

spkadd_status spkadd_tune(int32_t m, int32_t n, int32_t k, const int32_t* const* colptr, const int32_t* const* rowidx,
                          const void* const* values, spkadd_dtype dtype, const spkadd_opts* base, int32_t reps,
                          spkadd_opts* best, spkadd_tune_report* report, spkadd_tune_trial* trials,
                          int32_t max_trials, hipStream_t stream) {
  if (!best) return tfail(SPKADD_ERR_INVALID, "best is NULL");
  if (reps < 1 || reps > 100) return tfail(SPKADD_ERR_INVALID, "reps must be 1..100");
  if (max_trials < 0 || (max_trials > 0 && !trials)) return tfail(SPKADD_ERR_INVALID, "bad trials array");
  if (!values) return tfail(SPKADD_ERR_INVALID, "values is NULL");
  spkadd_opts o0;
  spkadd_opts_default(&o0);
  if (base) o0 = *base;

  // the inputs' size: one plan with the starting opts
  spkadd_stats stats{};
  {
    spkadd_plan_t p = nullptr;
    const spkadd_status st = spkadd_plan(&p, m, n, k, colptr, rowidx, dtype, &o0, stream);
    if (st != SPKADD_OK) return st;
    const spkadd_status s2 = spkadd_get_stats(p, &stats);
    spkadd_free(p);
    if (s2 != SPKADD_OK) return s2;
  }
  Runner R{m, n, k, colptr, rowidx, values, dtype, reps, stream};
  const size_t vb = dtype == SPKADD_F64 ? 8 : 4;
  const size_t cap = (size_t)std::max<long long>(stats.nnz_in, 1);
  if (hipMalloc((void**)&R.d_colptr, ((size_t)n + 1) * 4) != hipSuccess ||
      hipMalloc((void**)&R.d_rows, cap * 4) != hipSuccess || hipMalloc(&R.d_vals, cap * vb) != hipSuccess) {
    (void)hipGetLastError();
    if (R.d_colptr) (void)hipFree(R.d_colptr);
    if (R.d_rows) (void)hipFree(R.d_rows);
    return tfail(SPKADD_ERR_OOM, "tuner outputs (%zu entries)", cap);
  }
  R.got.assign((size_t)n + 1, 0);

  std::vector<Trial> done;
  auto run = [&](const spkadd_opts& o) -> const Trial& {
    Trial t;
    t.o = o;
    R.measure(t);
    done.push_back(t);
    return done.back();
  };
  auto usable = [](const Trial& t) { return t.st == SPKADD_OK && t.same && t.ms >= 0; };

  const Trial first = run(o0);
  if (first.st != SPKADD_OK) {
    (void)hipFree(R.d_colptr);
    (void)hipFree(R.d_rows);
    (void)hipFree(R.d_vals);
    return first.st;
  }
  spkadd_opts cur = o0;
  double cur_ms = first.ms;
  const bool long_cols = stats.n_wg_cols + stats.n_window_cols > 0;

  // one parameter at a time, every candidate value with the others fixed
  using Setter = void (*)(spkadd_opts&, double);
  struct Axis {
    Setter set;
    std::vector<double> values;
    bool long_only;
  };
  const std::vector<Axis> axes = {
      {[](spkadd_opts& o, double v) { o.wave_max = (int)v; }, {1024, 768, 512, 256}, false},
      {[](spkadd_opts& o, double v) {
         if (v < 0) {
           o.accum_mode = SPKADD_ACCUM_HASH;
         } else {
           o.accum_mode = SPKADD_ACCUM_AUTO;
           o.bitmap_ratio = (float)v;
         }
       },
       {1.0, 0.5, 2.0, 4.0, -1.0}, false},
      {[](spkadd_opts& o, double v) { o.wave_merge = (int)v; }, {0, 1}, false},
      {[](spkadd_opts& o, double v) { o.load_factor_sym = (float)v; }, {0.5, 0.35, 0.7}, false},
      {[](spkadd_opts& o, double v) { o.window_cap = (int)v; }, {0, 1024, 2048, 4096, 6144, 8192}, true},
      {[](spkadd_opts& o, double v) { o.window_fill = (float)v; }, {0.75, 0.5, 1.0}, true},
  };
  for (const Axis& ax : axes) {
    if (ax.long_only && !long_cols) continue;
    spkadd_opts axis_best = cur;
    double axis_ms = cur_ms;
    for (double v : ax.values) {
      spkadd_opts o = cur;
      ax.set(o, v);
      if (memcmp(&o, &cur, sizeof(o)) == 0) continue;  // the current setting
      const Trial& t = run(o);
      if (usable(t) && t.ms < axis_ms) {
        axis_ms = t.ms;
        axis_best = o;
      }
    }
    cur = axis_best;
    cur_ms = axis_ms;
  }
  (void)hipFree(R.d_colptr);
  (void)hipFree(R.d_rows);
  (void)hipFree(R.d_vals);

  *best = cur;
  spkadd_tune_key key{};
  spkadd_status st = spkadd_tune_key_for(m, n, k, stats.nnz_in, dtype, &key);
  if (st != SPKADD_OK) return st;
  st = spkadd_tune_store(&key, &cur, cur_ms);
  if (st != SPKADD_OK) return st;
  int failed = 0;
  for (const Trial& t : done) failed += !usable(t);
  if (report) {
    report->trials = (int32_t)done.size();
    report->failed = failed;
    report->default_ms = first.ms;
    report->best_ms = cur_ms;
    report->key = key;
  }
  for (int i = 0; i < (int)done.size() && i < max_trials; ++i) {
    trials[i].opts = done[i].o;
    trials[i].ms = done[i].ms;
    trials[i].status = (int32_t)done[i].st;
    trials[i].same_colptr = done[i].same ? 1 : 0;
  }
  return SPKADD_OK;
}

spkadd_status spkadd_tune_key_for_batch(int32_t nreq, int64_t sum_m, int64_t sum_n, int64_t sum_k, int64_t nnz_in,
                                        spkadd_dtype dtype, spkadd_tune_key* out) {
  if (!out) return tfail(SPKADD_ERR_INVALID, "out is NULL");
  if (nreq < 1 || sum_m < 0 || sum_n < 0 || sum_k < nreq || nnz_in < 0 || (dtype != SPKADD_F32 && dtype != SPKADD_F64))
    return tfail(SPKADD_ERR_INVALID, "bad request counts or dtype");
  spkadd_status st = spkadd_tune_key_for((int32_t)std::min<long long>(sum_m / nreq, INT32_MAX - 1),
                                         (int32_t)std::min<long long>(sum_n / nreq, INT32_MAX - 1),
                                         (int32_t)std::min<long long>((sum_k + nreq - 1) / nreq, INT32_MAX - 1), 0,
                                         dtype, out);
  if (st != SPKADD_OK) return st;
  out->u_log2 = sum_n > 0 ? ceil_log2_ll((nnz_in + sum_n - 1) / sum_n) : 0;
  out->kind = 1;
  return SPKADD_OK;
}

spkadd_status spkadd_tune_batch(const spkadd_request* reqs, int32_t nreq, spkadd_dtype dtype,
                                const spkadd_opts* base, int32_t reps, spkadd_opts* best,
                                spkadd_tune_report* report, spkadd_tune_trial* trials, int32_t max_trials,
                                hipStream_t stream) {
  if (!best || !reqs || nreq < 1) return tfail(SPKADD_ERR_INVALID, "NULL argument or no requests");
  if (reps < 1 || reps > 100) return tfail(SPKADD_ERR_INVALID, "reps must be 1..100");
  if (max_trials < 0 || (max_trials > 0 && !trials)) return tfail(SPKADD_ERR_INVALID, "bad trials array");
  spkadd_opts o0;
  spkadd_opts_default(&o0);
  if (base) o0 = *base;
  if (o0.batch_run_size <= 0) o0.batch_run_size = 8;
  // the sample's shape class: means of m, n, k and the input entries (colptr_i[n] of
  // every input, read from the device)
  long long sum_m = 0, sum_n = 0, sum_k = 0, nnz_in = 0;
  for (int r = 0; r < nreq; ++r) {
    const spkadd_request& q = reqs[r];
    if (!q.colptr || q.k < 1 || q.n < 0) return tfail(SPKADD_ERR_INVALID, "request %d is malformed", r);
    sum_m += q.m;
    sum_n += q.n;
    sum_k += q.k;
    for (int i = 0; i < q.k; ++i) {
      int32_t last = 0;
      if (!q.colptr[i] || hipMemcpy(&last, q.colptr[i] + q.n, 4, hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return tfail(SPKADD_ERR_INVALID, "request %d: colptr %d unreadable", r, i);
      }
      nnz_in += last;
    }
  }
  BatchRunner R{reqs, nreq, dtype, reps, stream};
  std::vector<Trial> done;
  auto run = [&](const spkadd_opts& o) -> const Trial& {
    Trial t;
    t.o = o;
    R.measure(t);
    done.push_back(t);
    return done.back();
  };
  auto usable = [](const Trial& t) { return t.st == SPKADD_OK && t.same && t.ms >= 0; };
  const Trial first = run(o0);
  if (first.st != SPKADD_OK) return first.st;
  spkadd_opts cur = o0;
  double cur_ms = first.ms;

  using Setter = void (*)(spkadd_opts&, double);
  struct Axis {
    Setter set;
    std::vector<double> values;
  };
  const std::vector<Axis> axes = {
      {[](spkadd_opts& o, double v) { o.batch_run_size = (int)v; }, {8, 16, 32, 64}},
      {[](spkadd_opts& o, double v) { o.batch_wave_max = (int)v; }, {1024, 768, 512}},
      {[](spkadd_opts& o, double v) { o.batch_wg_max = (int)v; }, {4096, 3072, 2048}},
      {[](spkadd_opts& o, double v) {
         if (v < 0) {
           o.accum_mode = SPKADD_ACCUM_HASH;
         } else {
           o.accum_mode = SPKADD_ACCUM_AUTO;
           o.bitmap_ratio = (float)v;
         }
       },
       {1.0, 0.5, 2.0, 4.0, -1.0}},
      {[](spkadd_opts& o, double v) { o.batch_fused_cols = (int)v; }, {0, -1}},
      {[](spkadd_opts& o, double v) { o.batch_wg_threads = (int)v; }, {256, 512}},
  };
  auto canon = [nreq](spkadd_opts o) {  // equal settings compare equal
    if (o.batch_wave_max == 0) o.batch_wave_max = 1024;
    if (o.batch_wg_max == 0) o.batch_wg_max = 4096;
    if (o.batch_wg_threads == 0) o.batch_wg_threads = 256;
    if (o.batch_run_size > nreq) o.batch_run_size = nreq;
    if (o.accum_mode == SPKADD_ACCUM_AUTO && o.bitmap_ratio == 0.f) o.bitmap_ratio = 1.f;
    return o;
  };
  for (const Axis& ax : axes) {
    spkadd_opts axis_best = cur;
    double axis_ms = cur_ms;
    for (double v : ax.values) {
      spkadd_opts o = cur;
      ax.set(o, v);
      const spkadd_opts a = canon(o), c = canon(cur);
      if (memcmp(&a, &c, sizeof(a)) == 0) continue;  // the current setting
      if (a.batch_wg_max < a.batch_wave_max) continue;  // no such setting
      if (o.batch_run_size > nreq) o.batch_run_size = nreq;
      const Trial& t = run(o);
      if (usable(t) && t.ms < axis_ms) {
        axis_ms = t.ms;
        axis_best = o;
      }
    }
    cur = axis_best;
    cur_ms = axis_ms;
  }
  if (cur.batch_run_size > nreq) cur.batch_run_size = nreq;
  *best = cur;
  spkadd_tune_key key{};
  spkadd_status st = spkadd_tune_key_for_batch(nreq, sum_m, sum_n, sum_k, nnz_in, dtype, &key);
  if (st != SPKADD_OK) return st;
  st = spkadd_tune_store(&key, &cur, cur_ms);
  if (st != SPKADD_OK) return st;
  int failed = 0;
  for (const Trial& t : done) failed += !usable(t);
  if (report) {
    report->trials = (int32_t)done.size();
    report->failed = failed;
    report->default_ms = first.ms;
    report->best_ms = cur_ms;
    report->key = key;
  }
  for (int i = 0; i < (int)done.size() && i < max_trials; ++i) {
    trials[i].opts = done[i].o;
    trials[i].ms = done[i].ms;
    trials[i].status = (int32_t)done[i].st;
    trials[i].same_colptr = done[i].same ? 1 : 0;
  }
  return SPKADD_OK;
}

spkadd_status spkadd_tune_lookup(const spkadd_tune_key* key, spkadd_opts* inout, int32_t* found) {
  if (!valid_key(key) || !inout || !found) return tfail(SPKADD_ERR_INVALID, "bad key or NULL argument");
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.entries.find(key_tuple(*key));
  *found = it != c.entries.end() ? 1 : 0;
  if (*found) apply(it->second, key->kind, *inout);
  return SPKADD_OK;
}

spkadd_status spkadd_tune_store(const spkadd_tune_key* key, const spkadd_opts* opts, double ms) {
  if (!valid_key(key) || !opts) return tfail(SPKADD_ERR_INVALID, "bad key or NULL opts");
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.entries[key_tuple(*key)] = tuned_of(*opts, ms);
  return SPKADD_OK;
}

int32_t spkadd_tune_size(void) {
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  return (int32_t)c.entries.size();
}

void spkadd_tune_clear(void) {
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.entries.clear();
}

spkadd_status spkadd_tune_save(const char* path) {
  if (!path) return tfail(SPKADD_ERR_INVALID, "path is NULL");
  std::string s = "{\"format\": \"spkadd-tune\", \"version\": 2, \"entries\": [";
  {
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    bool first = true;
    char buf[1024];
    for (auto& kv : c.entries) {
      const KeyTuple& k = kv.first;
      const Tuned& t = kv.second;
      s += first ? "\n  {" : ",\n  {";
      first = false;
      s += "\"arch\": ";
      put_str(s, std::get<0>(k));
      snprintf(buf, sizeof(buf),
               ", \"cus\": %d, \"dtype\": %d, \"m_log2\": %d, \"n_log2\": %d, \"k_log2\": %d, \"u_log2\": %d, "
               "\"kind\": %d, \"wave_max\": %d, \"accum_mode\": %d, \"bitmap_ratio\": %.9g, \"wave_merge\": %d, "
               "\"window_cap\": %d, \"load_factor_sym\": %.9g, \"load_factor_num\": %.9g, \"window_fill\": %.9g, "
               "\"batch_fused_cols\": %d, \"batch_wave_max\": %d, \"batch_wg_max\": %d, \"batch_wg_threads\": %d, "
               "\"batch_run_size\": %d, \"ms\": %.9g}",
               std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k),
               std::get<7>(k), t.wave_max, t.accum_mode, (double)t.bitmap_ratio, t.wave_merge, t.window_cap,
               (double)t.load_factor_sym, (double)t.load_factor_num, (double)t.window_fill, t.batch_fused_cols,
               t.batch_wave_max, t.batch_wg_max, t.batch_wg_threads, t.batch_run_size, t.ms);
      s += buf;
    }
  }
  s += "\n]}\n";
  FILE* f = fopen(path, "wb");
  if (!f) return tfail(SPKADD_ERR_STATE, "cannot write %s", path);
  const bool ok = fwrite(s.data(), 1, s.size(), f) == s.size();
  if (fclose(f) != 0 || !ok) return tfail(SPKADD_ERR_STATE, "cannot write %s", path);
  return SPKADD_OK;
}

spkadd_status spkadd_tune_load(const char* path) {
  if (!path) return tfail(SPKADD_ERR_INVALID, "path is NULL");
  FILE* f = fopen(path, "rb");
  if (!f) return tfail(SPKADD_ERR_STATE, "cannot read %s", path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, got);
    if (text.size() > (64u << 20)) {
      fclose(f);
      return tfail(SPKADD_ERR_INVALID, "%s: file too large", path);
    }
  }
  fclose(f);
  JParser P{text.data(), text.data() + text.size()};
  JVal root;
  if (!P.value(root)) return tfail(SPKADD_ERR_INVALID, "%s: not valid JSON", path);
  P.ws();
  if (P.p != P.end || root.kind != JVal::Obj) return tfail(SPKADD_ERR_INVALID, "%s: not a tuning cache", path);
  const JVal* fmt = root.get("format");
  const JVal* ver = root.get("version");
  const JVal* ents = root.get("entries");
  if (!fmt || fmt->kind != JVal::Str || fmt->str != "spkadd-tune" || !ver || ver->kind != JVal::Num ||
      (ver->num != 1 && ver->num != 2) || !ents || ents->kind != JVal::Arr)
    return tfail(SPKADD_ERR_INVALID, "%s: not a version 1 or 2 tuning cache", path);
  const bool v2 = ver->num == 2;
  std::vector<std::pair<KeyTuple, Tuned>> parsed;
  for (size_t i = 0; i < ents->arr.size(); ++i) {
    const JVal& e = ents->arr[i];
    const JVal* arch = e.kind == JVal::Obj ? e.get("arch") : nullptr;
    spkadd_tune_key key{};
    Tuned t;
    double d = 0;
    bool ok = arch && arch->kind == JVal::Str && arch->str.size() < sizeof(key.arch);
    if (ok) snprintf(key.arch, sizeof(key.arch), "%s", arch->str.c_str());
    ok = ok && int_field(e, "cus", 0, 1 << 20, &key.cus) && int_field(e, "dtype", 0, 1, &key.dtype) &&
         int_field(e, "m_log2", 0, 31, &key.m_log2) && int_field(e, "n_log2", 0, 31, &key.n_log2) &&
         int_field(e, "k_log2", 0, 31, &key.k_log2) && int_field(e, "u_log2", 0, 40, &key.u_log2) &&
         int_field(e, "wave_max", 0, 1024, &t.wave_max) && int_field(e, "accum_mode", 0, 2, &t.accum_mode) &&
         int_field(e, "wave_merge", 0, 1, &t.wave_merge) && int_field(e, "window_cap", 0, 8192, &t.window_cap);
    ok = ok && num_field(e, "bitmap_ratio", 0, 64, &d);
    t.bitmap_ratio = (float)d;
    ok = ok && num_field(e, "load_factor_sym", 0, 0.9, &d);
    t.load_factor_sym = (float)d;
    ok = ok && num_field(e, "load_factor_num", 0, 0.5, &d);
    t.load_factor_num = (float)d;
    ok = ok && num_field(e, "window_fill", 0, 1, &d);
    t.window_fill = (float)d;
    ok = ok && num_field(e, "ms", -1, 1e12, &t.ms);
    if (v2)  // version 2: the key's kind and the batch fields
      ok = ok && int_field(e, "kind", 0, 1, &key.kind) &&
           int_field(e, "batch_fused_cols", INT32_MIN, INT32_MAX, &t.batch_fused_cols) &&
           int_field(e, "batch_wave_max", 0, 1024, &t.batch_wave_max) &&
           int_field(e, "batch_wg_max", 0, 4096, &t.batch_wg_max) &&
           int_field(e, "batch_wg_threads", 0, 512, &t.batch_wg_threads) &&
           int_field(e, "batch_run_size", 0, 4096, &t.batch_run_size);
    if (!ok) return tfail(SPKADD_ERR_INVALID, "%s: entry %zu is malformed", path, i);
    parsed.emplace_back(key_tuple(key), t);
  }
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto& kv : parsed) c.entries[kv.first] = kv.second;
  return SPKADD_OK;
}

}  // extern "C"
