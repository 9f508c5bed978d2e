// Row windows over unsorted input columns (SPKADD_FLAG_UNSORTED_IN).  The sliding
// method (Section III-B, Algorithms 7-8) finds the entries of each window by binary
// search in sorted input columns.  Hash accumulation itself needs no order (Table I),
// so only the windows change: the entries of every window column are counted per
// window (a histogram against the column's window boundaries) to size and refine the
// windows, and once the windows are final they are partitioned into one contiguous
// bucket per window: the row, and the (input, position) of the entry, whose value the
// numeric pass gathers.  The window kernels then read a single input, the buckets.
#include "device.h"
#include "internal.h"

namespace spk {

constexpr int UW_THREADS = 256;
constexpr int UW_LDS_WIN = 4096;  // a column with at most this many windows counts / places them in LDS
constexpr int UW_LDS_K = 1024;    // at most this many inputs: one flat pass over the column's entries

// The window of `row` among a column's P windows, whose boundary rows are bro[0..P]
// (bro[0] = 0, bro[P] = m): the largest q < P with bro[q] <= row.
__device__ __forceinline__ int window_of(const int* __restrict__ bro, int P, int row) {
  int lo = 0, hi = P - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bro[mid] <= row) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One block per window column.  SCATTER = false: cnt[w] = entries of window w.
// SCATTER = true: each entry goes to slot cursor(w)++ of its window's bucket, which
// starts at boff[w] (cursors in LDS, or in `gcur`, preset to boff, for columns with
// more windows than LDS holds).
template <bool SCATTER>
__global__ __launch_bounds__(UW_THREADS) void k_uwin_pass(PlanParams p, const int* const* __restrict__ cp,
                                                        const int* const* __restrict__ ri,
                                                        const int* __restrict__ wcols, const int* __restrict__ wfirst,
                                                        const int* __restrict__ brow, int* __restrict__ cnt,
                                                        const int* __restrict__ boff, int* __restrict__ gcur,
                                                        int* __restrict__ brows, long long* __restrict__ bsrc) {
  __shared__ int segp[UW_LDS_K + 1];  // exclusive prefix of the segment lengths
  __shared__ int segs[UW_LDS_K];      // segment starts
  __shared__ int lc[UW_LDS_WIN];      // per-window counts or cursors
  __shared__ int red[UW_THREADS / 64 + 1];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int j = wcols[c], w0 = wfirst[c], P = wfirst[c + 1] - w0;
  const int* bro = brow + w0 + c;
  const bool lds_win = P <= UW_LDS_WIN;
  if (lds_win)
    for (int q = tid; q < P; q += UW_THREADS) lc[q] = SCATTER ? boff[w0 + q] : 0;
  auto place = [&](int i, int pos) {
    const int row = ri[i][pos];
    const int q = window_of(bro, P, row);
    if (!SCATTER) {
      atomicAdd(lds_win ? &lc[q] : &cnt[w0 + q], 1);
    } else {
      const int slot = atomicAdd(lds_win ? &lc[q] : &gcur[w0 + q], 1);
      brows[slot] = row;
      bsrc[slot] = ((long long)i << 32) | (unsigned)pos;
    }
  };
  if (p.k <= UW_LDS_K) {
    // one flat pass over the concatenated segments of all inputs
    int carry = 0;
    for (int base = 0; base < p.k; base += UW_THREADS) {
      const int i = base + tid;
      int s = 0, len = 0;
      if (i < p.k) {
        s = cp[i][j];
        len = max(cp[i][j + 1] - s, 0);
        segs[i] = s;
      }
      int chunk = 0;
      const int ex = block_excl_scan<UW_THREADS>(len, red, &chunk);
      if (i < p.k) segp[i] = carry + ex;
      carry += chunk;
    }
    if (tid == 0) segp[p.k] = carry;
    __syncthreads();
    int ktop = 0;  // largest power of two <= k - 1
    while ((ktop << 1) <= p.k - 1) ktop = ktop ? ktop << 1 : 1;
    if (p.k == 1) ktop = 0;
    for (int e = tid; e < carry; e += UW_THREADS) {
      int lo = 0;
      for (int step = ktop; step > 0; step >>= 1)
        if (lo + step < p.k && segp[lo + step] <= e) lo += step;
      place(lo, segs[lo] + (e - segp[lo]));
    }
  } else {
    __syncthreads();
    for (int i = 0; i < p.k; ++i) {
      const int s = cp[i][j], e = cp[i][j + 1];
      for (int pos = s + tid; pos < e; pos += UW_THREADS) place(i, pos);
    }
  }
  if (!SCATTER && lds_win) {
    __syncthreads();
    for (int q = tid; q < P; q += UW_THREADS) cnt[w0 + q] = lc[q];
  }
}

// Boundary positions of the buckets, in the layout the window kernels read for one
// input: bpos[w + c] = start of window w's bucket, and after a column's last window
// its end.
__global__ __launch_bounds__(256) void k_uwin_bpos(int n_windows, const int* __restrict__ win_c,
                                                   const int* __restrict__ wfirst, const int* __restrict__ boff,
                                                   int* __restrict__ bpos) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= n_windows) return;
  const int c = win_c[w];
  bpos[w + c] = boff[w];
  if (w + 1 == wfirst[c + 1]) bpos[w + c + 1] = boff[w + 1];
}

// Values of the bucket entries for one numeric pass.
template <typename V>
__global__ __launch_bounds__(256) void k_uwin_gather(long long total, const long long* __restrict__ bsrc,
                                                     const void* const* __restrict__ va, V* __restrict__ bvals) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const long long s = bsrc[t];
  bvals[t] = reinterpret_cast<const V*>(va[(int)(s >> 32)])[(unsigned)s];
}

void launch_uwin_hist(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int n_wcols,
                      const int* d_wcols, const int* d_wfirst, const int* d_brow, int* d_cnt, hipStream_t s) {
  if (n_wcols <= 0) return;
  k_uwin_pass<false><<<n_wcols, UW_THREADS, 0, s>>>(p, d_cp, d_ri, d_wcols, d_wfirst, d_brow, d_cnt, nullptr,
                                                    nullptr, nullptr, nullptr);
}

void launch_uwin_scatter(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int n_wcols,
                         const int* d_wcols, const int* d_wfirst, const int* d_brow, const int* d_boff, int* d_gcur,
                         int* d_brows, long long* d_bsrc, hipStream_t s) {
  if (n_wcols <= 0) return;
  k_uwin_pass<true><<<n_wcols, UW_THREADS, 0, s>>>(p, d_cp, d_ri, d_wcols, d_wfirst, d_brow, nullptr, d_boff,
                                                   d_gcur, d_brows, d_bsrc);
}

void launch_uwin_bpos(int n_windows, const int* d_win_c, const int* d_wfirst, const int* d_boff, int* d_bpos,
                      hipStream_t s) {
  if (n_windows <= 0) return;
  k_uwin_bpos<<<(n_windows + 255) / 256, 256, 0, s>>>(n_windows, d_win_c, d_wfirst, d_boff, d_bpos);
}

void launch_uwin_gather(long long total, const long long* d_bsrc, const void* const* d_va, void* d_bvals, bool f64,
                        hipStream_t s) {
  if (total <= 0) return;
  const unsigned grid = (unsigned)((total + 255) / 256);
  if (f64) k_uwin_gather<double><<<grid, 256, 0, s>>>(total, d_bsrc, d_va, (double*)d_bvals);
  else k_uwin_gather<float><<<grid, 256, 0, s>>>(total, d_bsrc, d_va, (float*)d_bvals);
}

}  // namespace spk
