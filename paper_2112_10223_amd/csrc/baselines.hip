// The k-way heap merge of Algorithm 3 (HeapAdd, Section II-C) on the GPU, as the
// baseline the hash method is measured against (include/spkadd_baselines.h): one
// thread per column, the column's min-heap of (row, input) in LDS.  Symbolic pass:
// distinct rows per column; scan: colptr(B); numeric pass: the merged column.
#include <climits>
#include <vector>

#include "device.h"
#include "internal.h"
#include "spkadd_baselines.h"

namespace spk {

constexpr int HEAP_THREADS = 64;

struct HeapArgs {
  int n, k;
  const int* const* cp;
  const int* const* ri;
  const void* const* va;
  int* colcnt;          // symbolic: distinct rows per column
  const int* colptr_c;  // numeric: colptr(B)
  int* out_r;
  void* out_v;
};

// LDS per thread: heap rows, heap inputs, and each input's cursor and end (k each).
template <bool NUM, typename V>
__global__ __launch_bounds__(HEAP_THREADS) void k_heap(HeapArgs h) {
  extern __shared__ int hs[];
  const int t = threadIdx.x, K = h.k;
  const int j = blockIdx.x * HEAP_THREADS + t;
  if (j >= h.n) return;  // (no barriers below)
  int* hrow = hs + t * K;
  int* hin = hs + (HEAP_THREADS + t) * K;
  int* pos = hs + (2 * HEAP_THREADS + t) * K;
  int* end = hs + (3 * HEAP_THREADS + t) * K;
  // the heap of every input's first entry
  int sz = 0;
  for (int i = 0; i < K; ++i) {
    const int s = h.cp[i][j], e = h.cp[i][j + 1];
    pos[i] = s;
    end[i] = e;
    if (s < e) {
      const int r = h.ri[i][s];
      int c = sz++;
      while (c > 0) {
        const int par = (c - 1) >> 1;
        if (hrow[par] <= r) break;
        hrow[c] = hrow[par];
        hin[c] = hin[par];
        c = par;
      }
      hrow[c] = r;
      hin[c] = i;
    }
  }
  int cnt = 0, last = -1;
  const int o = NUM ? h.colptr_c[j] : 0;
  int* out_r = h.out_r;
  V* out_v = reinterpret_cast<V*>(h.out_v);
  V acc = V(0);
  while (sz > 0) {
    const int r = hrow[0], i = hin[0];
    if (r != last) {
      if (NUM && cnt > 0) {
        out_r[o + cnt - 1] = last;
        out_v[o + cnt - 1] = acc;
      }
      ++cnt;
      last = r;
      if (NUM) acc = reinterpret_cast<const V*>(h.va[i])[pos[i]];
    } else if (NUM) {
      acc += reinterpret_cast<const V*>(h.va[i])[pos[i]];
    }
    // the next entry of input i replaces the top, or the last heap entry does
    const int p = ++pos[i];
    int nr, ni;
    if (p < end[i]) {
      nr = h.ri[i][p];
      ni = i;
    } else {
      if (--sz == 0) break;
      nr = hrow[sz];
      ni = hin[sz];
    }
    int c = 0;
    for (;;) {
      int ch = 2 * c + 1;
      if (ch >= sz) break;
      if (ch + 1 < sz && hrow[ch + 1] < hrow[ch]) ++ch;
      if (hrow[ch] >= nr) break;
      hrow[c] = hrow[ch];
      hin[c] = hin[ch];
      c = ch;
    }
    hrow[c] = nr;
    hin[c] = ni;
  }
  if (NUM) {
    if (cnt > 0) {
      out_r[o + cnt - 1] = last;
      out_v[o + cnt - 1] = acc;
    }
  } else {
    h.colcnt[j] = cnt;
  }
}

static hipError_t launch_heap(bool numeric, bool f64, const HeapArgs& h, hipStream_t s) {
  const unsigned grid = (unsigned)((h.n + HEAP_THREADS - 1) / HEAP_THREADS);
  const size_t lds = (size_t)4 * HEAP_THREADS * h.k * sizeof(int);
  if (!numeric) k_heap<false, float><<<grid, HEAP_THREADS, lds, s>>>(h);
  else if (f64) k_heap<true, double><<<grid, HEAP_THREADS, lds, s>>>(h);
  else k_heap<true, float><<<grid, HEAP_THREADS, lds, s>>>(h);
  return hipGetLastError();
}

}  // namespace spk

namespace {
spkadd_status heap_error(spkadd_status st, const char* msg) { return spk::report_error(st, msg); }
}  // namespace

extern "C" spkadd_status spkadd_heap_add(int32_t m, int32_t n, int32_t k, const int32_t* const* colptr,
                                         const int32_t* const* rowidx, const void* const* values, spkadd_dtype dtype,
                                         int32_t* colptr_c, int32_t* rowidx_c, void* values_c, int64_t cap_c,
                                         int64_t* nnz_c, hipStream_t stream) {
  using namespace spk;
  spk::report_error(SPKADD_OK, "");
  if (m < 0 || n < 0 || m == INT_MAX || n == INT_MAX) return heap_error(SPKADD_ERR_INVALID, "bad shape");
  if (k < 1 || k > SPKADD_HEAP_MAX_K) return heap_error(SPKADD_ERR_INVALID, "k must be in [1, SPKADD_HEAP_MAX_K]");
  if (!colptr || !rowidx || !values || !colptr_c || !nnz_c || cap_c < 0)
    return heap_error(SPKADD_ERR_INVALID, "NULL argument or negative capacity");
  if (dtype != SPKADD_F32 && dtype != SPKADD_F64) return heap_error(SPKADD_ERR_INVALID, "bad dtype");
  for (int i = 0; i < k; ++i)
    if (!colptr[i]) return heap_error(SPKADD_ERR_INVALID, "colptr[i] is NULL");
  if (cap_c > 0 && (!rowidx_c || !values_c)) return heap_error(SPKADD_ERR_INVALID, "NULL output arrays");
  // device workspace: pointer tables, column counts, scan scratch, total and flags
  std::vector<const void*> tab(3 * (size_t)k);
  for (int i = 0; i < k; ++i) {
    tab[i] = colptr[i];
    tab[k + i] = rowidx[i];
    tab[2 * k + i] = values[i];
  }
  const size_t o_tab = 0, o_cnt = (3 * (size_t)k * 8 + 255) & ~(size_t)255;
  const size_t o_tot = (o_cnt + (size_t)n * 4 + 255) & ~(size_t)255, o_tmp = o_tot + 256;
  const size_t bytes = o_tmp + scan_tmp_bytes(n);
  char* ws = nullptr;
  if (hipMallocAsync((void**)&ws, bytes, stream) != hipSuccess) {
    (void)hipGetLastError();
    return heap_error(SPKADD_ERR_OOM, "workspace allocation failed");
  }
  auto fail_hip = [&](const char* what) {
    (void)hipGetLastError();
    (void)hipFreeAsync(ws, stream);
    return heap_error(SPKADD_ERR_HIP, what);
  };
  long long* d_tot = (long long*)(ws + o_tot);
  int* d_err = (int*)(ws + o_tot + 8);
  if (hipMemcpyAsync(ws + o_tab, tab.data(), tab.size() * sizeof(void*), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipMemsetAsync(d_err, 0, sizeof(int), stream) != hipSuccess)
    return fail_hip("workspace upload failed");
  HeapArgs h{};
  h.n = n;
  h.k = k;
  h.cp = (const int* const*)(ws + o_tab);
  h.ri = (const int* const*)(ws + o_tab + (size_t)k * 8);
  h.va = (const void* const*)(ws + o_tab + 2 * (size_t)k * 8);
  h.colcnt = (int*)(ws + o_cnt);
  if (n > 0 && launch_heap(false, false, h, stream) != hipSuccess) return fail_hip("heap symbolic launch failed");
  launch_scan(h.colcnt, n, colptr_c, d_tot, d_err, ws + o_tmp, stream);
  long long total = 0;
  int err = 0;
  if (hipMemcpyAsync(&total, d_tot, sizeof(total), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(&err, d_err, sizeof(err), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail_hip("count readback failed");
  *nnz_c = total;
  if (err || total > INT_MAX) {
    (void)hipFreeAsync(ws, stream);
    return heap_error(SPKADD_ERR_OVERFLOW, "nnz(B) exceeds INT32_MAX");
  }
  if (total > 0 && total <= cap_c) {
    h.colptr_c = colptr_c;
    h.out_r = rowidx_c;
    h.out_v = values_c;
    if (launch_heap(true, dtype == SPKADD_F64, h, stream) != hipSuccess) return fail_hip("heap numeric launch failed");
  }
  (void)hipFreeAsync(ws, stream);
  return SPKADD_OK;
}
