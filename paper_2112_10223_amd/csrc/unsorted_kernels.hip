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
constexpr int UW_LDS_WIN = 4096;  // a column with at most this many windows counts them in LDS
constexpr int UW_LDS_K = WIN_LDS_K;  // at most this many inputs: one flat pass over the column's entries

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

// Work units of the window passes: chunks of UW_CHUNK entries of a column's
// concatenated input segments (one chunk per column when it has more inputs than the
// on-chip segment table), so that a long column is spread over many workgroups.
constexpr int UW_CHUNK = WIN_CHUNK;
constexpr int UW_EPT = UW_CHUNK / UW_THREADS;  // entries of a chunk per thread, kept in registers

__global__ __launch_bounds__(256) void k_uwin_nch(PlanParams p, int n_wcols, const int* __restrict__ wcols,
                                                  const int* __restrict__ u, int chunk,
                                                  const int* __restrict__ wlin, int* __restrict__ nch) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_wcols) return;
  const int uc = u[wcols[c]];
  nch[c] = wlin && wlin[c] ? 0
           : p.k <= UW_LDS_K                         ? max((int)(((long long)uc + chunk - 1) / chunk), 1)
                                                     : 1;
}

__global__ __launch_bounds__(256) void k_uwin_chfill(int n_wcols, const int* __restrict__ chfirst,
                                                     int* __restrict__ chcol) {
  const int c = blockIdx.x;
  if (c >= n_wcols) return;
  for (int t = chfirst[c] + threadIdx.x; t < chfirst[c + 1]; t += 256) chcol[t] = c;
}

// One workgroup per chunk.  SCATTER = false: cnt[w] += entries of window w in the
// chunk.  SCATTER = true: the chunk reserves a range of each window's bucket (gcur:
// the next free slot of each bucket, preset to its start) and places its entries
// there: the row and the entry's (input, position).  Windows are counted in LDS
// when the column has at most UW_LDS_WIN of them, else by global atomics per entry.
template <bool SCATTER>
__global__ __launch_bounds__(UW_THREADS) void k_uwin_pass(PlanParams p, const int* const* __restrict__ cp,
                                                        const int* const* __restrict__ ri,
                                                        const int* __restrict__ wcols, const int* __restrict__ wfirst,
                                                        const int* __restrict__ brow,
                                                        const int* __restrict__ chfirst,
                                                        const int* __restrict__ chcol, int* __restrict__ cnt,
                                                        int* __restrict__ gcur, int* __restrict__ brows,
                                                        long long* __restrict__ bsrc) {
  __shared__ int segp[UW_LDS_K + 1];  // exclusive prefix of the segment lengths
  __shared__ int segs[UW_LDS_K];      // segment starts
  __shared__ int lc[UW_LDS_WIN];      // per-window counts, then cursors
  __shared__ int lbro[UW_LDS_WIN + 1];
  __shared__ int red[UW_THREADS / 64 + 1];
  const int tid = threadIdx.x;
  const int c = chcol[blockIdx.x], chunk = blockIdx.x - chfirst[c];
  const int j = wcols[c], w0 = wfirst[c], P = wfirst[c + 1] - w0;
  const int* bro = brow + w0 + c;
  const bool lds_win = P <= UW_LDS_WIN;
  if (lds_win) {
    for (int q = tid; q <= P; q += UW_THREADS) lbro[q] = bro[q];
    for (int q = tid; q < P; q += UW_THREADS) lc[q] = 0;
  }
  auto win = [&](int row) { return lds_win ? window_of(lbro, P, row) : window_of(bro, P, row); };
  auto put = [&](int slot, int row, int i, int pos) {
    brows[slot] = row;
    bsrc[slot] = ((long long)i << 32) | (unsigned)pos;
  };
  // the first pass counts (or, without LDS counters, does all the work); the second
  // places the entries of an LDS-counted chunk
  auto first = [&](int i, int pos) {
    const int row = ri[i][pos];
    const int q = win(row);
    if (lds_win) atomicAdd(&lc[q], 1);
    else if (!SCATTER) atomicAdd(&cnt[w0 + q], 1);
    else put(atomicAdd(&gcur[w0 + q], 1), row, i, pos);
  };
  auto second = [&](int i, int pos) {
    const int row = ri[i][pos];
    put(atomicAdd(&lc[win(row)], 1), row, i, pos);
  };
  if (p.k <= UW_LDS_K) {
    // the column's entries as one concatenated range; this chunk is [e0, e1)
    int carry = 0;
    for (int base = 0; base < p.k; base += UW_THREADS) {
      const int i = base + tid;
      int s = 0, len = 0;
      if (i < p.k) {
        s = cp[i][j];
        len = max(cp[i][j + 1] - s, 0);
        segs[i] = s;
      }
      int chunk_sum = 0;
      const int ex = block_excl_scan<UW_THREADS>(len, red, &chunk_sum);
      if (i < p.k) segp[i] = carry + ex;
      carry += chunk_sum;
    }
    if (tid == 0) segp[p.k] = carry;
    __syncthreads();
    int ktop = 0;  // largest power of two <= k - 1
    while ((ktop << 1) <= p.k - 1) ktop = ktop ? ktop << 1 : 1;
    if (p.k == 1) ktop = 0;
    const long long e0l = (long long)chunk * UW_CHUNK;
    const int e0 = (int)(e0l < carry ? e0l : carry);
    const int e1 = (int)(e0l + UW_CHUNK < carry ? e0l + UW_CHUNK : carry);
    // every entry of the chunk once: row, window and source kept in registers for the
    // placement after the reservation (clamped index: no guard on the loads)
    int rowv[UW_EPT], qv[UW_EPT], iv[UW_EPT], posv[UW_EPT];
    if (e0 < e1) {  // (uniform)
#pragma unroll
      for (int t = 0; t < UW_EPT; ++t) {
        const int e = min(e0 + tid + t * UW_THREADS, e1 - 1);
        int lo = 0;
        for (int step = ktop; step > 0; step >>= 1)
          if (lo + step < p.k && segp[lo + step] <= e) lo += step;
        iv[t] = lo;
        posv[t] = segs[lo] + (e - segp[lo]);
        rowv[t] = ri[lo][posv[t]];
      }
#pragma unroll
      for (int t = 0; t < UW_EPT; ++t) {
        const bool mine = e0 + tid + t * UW_THREADS < e1;
        qv[t] = mine ? win(rowv[t]) : -1;
        if (!mine) continue;
        if (lds_win) atomicAdd(&lc[qv[t]], 1);
        else if (!SCATTER) atomicAdd(&cnt[w0 + qv[t]], 1);
        else put(atomicAdd(&gcur[w0 + qv[t]], 1), rowv[t], iv[t], posv[t]);
      }
    }
    __syncthreads();
    if (lds_win) {
      if (!SCATTER) {
        for (int q = tid; q < P; q += UW_THREADS)
          if (lc[q]) atomicAdd(&cnt[w0 + q], lc[q]);
      } else {
        for (int q = tid; q < P; q += UW_THREADS)
          if (lc[q]) lc[q] = atomicAdd(&gcur[w0 + q], lc[q]);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < UW_EPT; ++t)
          if (qv[t] >= 0) put(atomicAdd(&lc[qv[t]], 1), rowv[t], iv[t], posv[t]);
      }
    }
  } else {
    // more inputs than the segment table: one chunk per column, input by input
    __syncthreads();
    for (int i = 0; i < p.k; ++i) {
      const int s = cp[i][j], e = cp[i][j + 1];
      for (int pos = s + tid; pos < e; pos += UW_THREADS) first(i, pos);
    }
    __syncthreads();
    if (lds_win) {
      if (!SCATTER) {
        for (int q = tid; q < P; q += UW_THREADS)
          if (lc[q]) atomicAdd(&cnt[w0 + q], lc[q]);
      } else {
        for (int q = tid; q < P; q += UW_THREADS)
          if (lc[q]) lc[q] = atomicAdd(&gcur[w0 + q], lc[q]);
        __syncthreads();
        for (int i = 0; i < p.k; ++i) {
          const int s = cp[i][j], e = cp[i][j + 1];
          for (int pos = s + tid; pos < e; pos += UW_THREADS) second(i, pos);
        }
      }
    }
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

void launch_uwin_chunks(const PlanParams& p, int n_wcols, const int* d_wcols, const int* d_u, int chunk,
                        const int* d_wlin, int* d_nch, hipStream_t s) {
  if (n_wcols <= 0) return;
  k_uwin_nch<<<(n_wcols + 255) / 256, 256, 0, s>>>(p, n_wcols, d_wcols, d_u, chunk, d_wlin, d_nch);
}

void launch_uwin_chfill(int n_wcols, const int* d_chfirst, int* d_chcol, hipStream_t s) {
  if (n_wcols <= 0) return;
  k_uwin_chfill<<<n_wcols, 256, 0, s>>>(n_wcols, d_chfirst, d_chcol);
}

void launch_uwin_hist(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int n_chunks,
                      const int* d_wcols, const int* d_wfirst, const int* d_brow, const int* d_chfirst,
                      const int* d_chcol, int* d_cnt, hipStream_t s) {
  if (n_chunks <= 0) return;
  k_uwin_pass<false><<<n_chunks, UW_THREADS, 0, s>>>(p, d_cp, d_ri, d_wcols, d_wfirst, d_brow, d_chfirst, d_chcol,
                                                     d_cnt, nullptr, nullptr, nullptr);
}

void launch_uwin_scatter(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int n_chunks,
                         const int* d_wcols, const int* d_wfirst, const int* d_brow, const int* d_chfirst,
                         const int* d_chcol, int* d_gcur, int* d_brows, long long* d_bsrc, hipStream_t s) {
  if (n_chunks <= 0) return;
  k_uwin_pass<true><<<n_chunks, UW_THREADS, 0, s>>>(p, d_cp, d_ri, d_wcols, d_wfirst, d_brow, d_chfirst, d_chcol,
                                                    nullptr, d_gcur, d_brows, d_bsrc);
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
