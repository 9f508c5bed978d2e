// Planning kernels: per-column upper bounds and bins (the load balance of
// Section III-A), the row windows of the sliding hash (Section III-B), and scans.
#include <climits>

#include "device.h"
#include "internal.h"
#include "scan_device.h"

namespace spk {

__device__ __forceinline__ int classify(long long u, const PlanParams& p) {
  if (u <= 0) return BIN_EMPTY;
  if (p.force_bin == 2) return BIN_WIN;
  if (p.force_bin == 1) {
    if (u <= p.cap_in) return u <= p.g1_max ? BIN_G1 : BIN_G2;
    return BIN_WIN;
  }
  const int wave_limit = p.force_bin == 0 ? 1024 : p.wave_max;
  if (u <= wave_limit) {
    const int e = (int)((u + 63) >> 6);
    return e <= 1 ? BIN_W1 : e <= 2 ? BIN_W2 : e <= 3 ? BIN_W3 : e <= 4 ? BIN_W4 : e <= 5 ? BIN_W5
         : e <= 6 ? BIN_W6 : e <= 8 ? BIN_W8 : e <= 10 ? BIN_W10 : e <= 12 ? BIN_W12 : BIN_W16;
  }
  if (u <= p.cap_in) return u <= p.g1_max ? BIN_G1 : BIN_G2;
  return BIN_WIN;
}

// u_j = sum_i nnz(A_i(:,j)), bin of j, per-block bin histogram, nnz_in.
__global__ __launch_bounds__(PLAN_THREADS) void k_bounds(PlanParams p, const int* const* __restrict__ cp,
                                                         const int* const* __restrict__ ri, int* __restrict__ u, unsigned char* __restrict__ bin,
                                                         int* __restrict__ colcnt, int* __restrict__ hist,
                                                         PlanSummary* __restrict__ sum) {
  __shared__ int wh[PLAN_THREADS / 64][NBINS];
  __shared__ unsigned long long red[PLAN_THREADS / 64 + 1];
  if (blockIdx.x == 0)  // an input with entries must come with a row array
    for (int i = threadIdx.x; i < p.k; i += PLAN_THREADS)
      if (cp[i][p.n] > 0 && ri[i] == nullptr) atomicOr(&sum->err, ERR_INPUT);
  const int j = blockIdx.x * PLAN_THREADS + threadIdx.x;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  long long uj = 0;
  int b = -1;
  if (j < p.n) {
    // 16 inputs per round, all their loads in flight before the first is used (the
    // loop is bound by memory latency, not bandwidth: one column per thread)
    for (int i0 = 0; i0 < p.k; i0 += 16) {
      long long ptr[16];
      int s[16], e[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) ptr[t] = (long long)cp[min(i0 + t, p.k - 1)];
      // (global loads: through a generic pointer they would share the scalar loads'
      // wait counter and be waited for one by one)
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        s[t] = gload<int>(ptr[t] + 4LL * j);
        e[t] = gload<int>(ptr[t] + 4LL * (j + 1));
      }
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (i0 + t < p.k) uj += (long long)(e[t] - s[t]);
    }
    if (uj > INT_MAX) {
      atomicOr(&sum->err, ERR_OVERFLOW);
      uj = INT_MAX;
    }
    b = classify(uj, p);
    u[j] = (int)uj;
    bin[j] = (unsigned char)b;
    colcnt[j] = 0;
  }
  for (int bb = 0; bb < NBINS; ++bb) {
    const uint64_t mk = ballot(b == bb);
    if (lane == 0) wh[w][bb] = __popcll(mk);
  }
  const unsigned long long tot = block_sum<PLAN_THREADS>((unsigned long long)uj, red);
  if (threadIdx.x < NBINS) {
    int s = 0;
    for (int v = 0; v < PLAN_THREADS / 64; ++v) s += wh[v][threadIdx.x];
    hist[blockIdx.x * NBINS + threadIdx.x] = s;
  }
  if (threadIdx.x == 0 && tot) atomicAdd(&sum->nnz_in, tot);
}

// Optional input validation: colptr_i[0] = 0, colptr non-decreasing, rows in [0, m)
// and (unless the input is declared unsorted) strictly ascending within every column.
__global__ __launch_bounds__(PLAN_THREADS) void k_validate(PlanParams p, const int* const* __restrict__ cp,
                                                           const int* const* __restrict__ ri,
                                                           PlanSummary* __restrict__ sum) {
  const int j = blockIdx.x * PLAN_THREADS + threadIdx.x;
  if (j >= p.n) return;
  bool bad = false;
  for (int i = 0; i < p.k; ++i) {
    const int* c = cp[i];
    const int s = c[j], e = c[j + 1];
    if (j == 0 && s != 0) bad = true;
    if (e < s || s < 0) {
      bad = true;
      continue;
    }
    const int* r = ri[i];
    int prev = -1;
    for (int q = s; q < e; ++q) {
      const int row = r[q];
      if ((!p.unsorted_in && row <= prev) || row < 0 || row >= p.m) bad = true;
      prev = row;
    }
  }
  if (bad) atomicOr(&sum->err, ERR_INPUT);
}

// Copies a chunk of device pointers, passed by value, into a device table; the
// first chunk of a plan also clears the plan summary and the dummy buffer.
__global__ __launch_bounds__(256) void k_put_ptrs(PtrChunk c, const void** __restrict__ dst,
                                                  PlanSummary* __restrict__ sum, unsigned* __restrict__ dummy) {
  const int t = threadIdx.x;
  if (t < c.count) dst[t] = c.p[t];
  if (sum)
    for (int i = t; i < (int)(sizeof(PlanSummary) / 4); i += 256) reinterpret_cast<int*>(sum)[i] = 0;
  if (dummy)
    for (int i = t; i < 1024; i += 256) dummy[i] = 0u;
}

// Exclusive scan, over blocks, of the per-block bin histograms; bin offsets; bin
// counts into the summary.  One block of 1024 threads.
//
// Wave-bin merging: each input column's rows are only a few dozen bytes, less than
// a cache line, and neighbouring columns share lines.  When a column population is
// split between two adjacent wave bins (as a Poisson column length around a bin
// edge is), the two kernels fetch the shared lines twice.  With merge set, two
// adjacent non-empty wave bins that each hold at least 1/16 of the wave columns,
// and whose E differ by at most 3/2, become one bin (the larger E); a column of
// the smaller bin then runs with some lanes idle.  binoff[NBINS + 1 + b] receives
// the bin that bin b's columns go to.
__global__ __launch_bounds__(1024) void k_bin_scan(int nblk, int merge, int* __restrict__ hist,
                                                   int* __restrict__ binoff, PlanSummary* __restrict__ sum) {
  static_assert(NBINS <= 1024 / 64, "one wavefront per bin");
  __shared__ int totals[NBINS];
  __shared__ int map[NBINS];
  __shared__ int mtot[NBINS];
  const int lane = lane_id(), b = threadIdx.x >> 6;
  if (b < NBINS) {
    int s = 0;
    for (int base = 0; base < nblk; base += 64) {
      const int t = base + lane;
      s += t < nblk ? hist[t * NBINS + b] : 0;
    }
    s = wave_total_add(s);
    if (lane == 0) totals[b] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int x = 0; x < NBINS; ++x) map[x] = x;
    if (merge) {
      long long wave_cols = 0;
      for (int x = BIN_W1; x <= BIN_W16; ++x) wave_cols += totals[x];
      int prev = -1;
      for (int x = BIN_W1; x <= BIN_W16; ++x) {
        if (totals[x] == 0) continue;
        if (prev >= 0 && 16LL * totals[prev] >= wave_cols && 16LL * totals[x] >= wave_cols &&
            2 * wave_bin_E(x) <= 3 * wave_bin_E(prev)) {
          map[prev] = x;  // pairs only: x takes no further merge
          prev = -1;
        } else {
          prev = x;
        }
      }
    }
  }
  __syncthreads();
  // wavefront b scans, over blocks, the per-block counts of the bins mapped to b
  if (b < NBINS && map[b] == b) {
    int carry = 0;
    for (int base = 0; base < nblk; base += 64) {
      const int t = base + lane;
      int v = 0;
      if (t < nblk)
        for (int x = 0; x < NBINS; ++x) v += map[x] == b ? hist[t * NBINS + x] : 0;
      const int incl = wave_scan_add(v);
      if (t < nblk) hist[t * NBINS + b] = carry + incl - v;
      carry += readlane(incl, 63);
    }
    if (lane == 0) mtot[b] = carry;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int bb = 0; bb < NBINS; ++bb) {
      const int c = map[bb] == bb ? mtot[bb] : 0;
      binoff[bb] = acc;
      binoff[NBINS + 1 + bb] = map[bb];
      sum->bin_count[bb] = c;
      acc += c;
    }
    binoff[NBINS] = acc;
  }
}

// Column ids grouped by bin, in column order inside each bin.
__global__ __launch_bounds__(PLAN_THREADS) void k_bin_scatter(PlanParams p, const unsigned char* __restrict__ bin,
                                                              const int* __restrict__ hist,
                                                              const int* __restrict__ binoff,
                                                              int* __restrict__ list) {
  __shared__ int wc[PLAN_THREADS / 64][NBINS];
  const int j = blockIdx.x * PLAN_THREADS + threadIdx.x;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int b = j < p.n ? binoff[NBINS + 1 + (int)bin[j]] : -1;  // bin after merging
  int rank = 0;
  for (int bb = 0; bb < NBINS; ++bb) {
    const uint64_t mk = ballot(b == bb);
    if (b == bb) rank = mbcnt(mk);
    if (lane == 0) wc[w][bb] = __popcll(mk);
  }
  __syncthreads();
  if (b > BIN_EMPTY) {
    int before = 0;
    for (int v = 0; v < w; ++v) before += wc[v][b];
    list[binoff[b] + hist[blockIdx.x * NBINS + b] + before + rank] = j;
  }
}

// Initial number of windows of each window column: P = ceil(u / (cap_in * fill)), at
// least win_min, clamped to [1, m]; exclusive scan into wfirst[0..n_wcols].  One block.
__global__ __launch_bounds__(1024) void k_win_scan(PlanParams p, const int* __restrict__ list,
                                                   const int* __restrict__ binoff, const int* __restrict__ u,
                                                   int* __restrict__ wfirst, PlanSummary* __restrict__ sum) {
  __shared__ long long scratch[1024 / 64 + 1];
  const int* wcols = list + binoff[BIN_WIN];
  const int n_wcols = binoff[BIN_WIN + 1] - binoff[BIN_WIN];
  const double target = (double)p.cap_in * (double)p.win_fill;
  long long carry = 0;
  for (int base = 0; base < n_wcols; base += 1024) {
    const int c = base + threadIdx.x;
    long long pc = 0;
    if (c < n_wcols) {
      const int uj = u[wcols[c]];
      pc = (long long)ceil((double)uj / (target > 1.0 ? target : 1.0));
      if (pc < p.win_min) pc = p.win_min;
      if (pc < 1) pc = 1;
      if (pc > p.m) pc = p.m;
    }
    long long chunk = 0;
    const long long ex = block_excl_scan<1024>(pc, scratch, &chunk);
    if (c < n_wcols) wfirst[c] = (int)(carry + ex);
    carry += chunk;
  }
  if (threadIdx.x == 0) {
    if (carry > (long long)(INT_MAX / 2)) {
      atomicOr(&sum->err, ERR_OVERFLOW);
      carry = 0;
    }
    wfirst[n_wcols] = (int)carry;
    sum->n_windows = (int)carry;
  }
}

__device__ __forceinline__ int lower_bound_rows(const int* __restrict__ r, int lo, int hi, int row) {
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if (r[mid] < row) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// First windows of each window column.  The paper splits a column's rows equally
// (Algorithms 7-8: window q covers rows [q m / P, (q + 1) m / P)), and so do the
// columns of the ordered pass (win_search_linear).  Elsewhere, where the inputs are
// sorted, the boundaries are instead the row quantiles of the column's longest input (the row at
// position floor(q len / P) of that input's column): for inputs of similar row
// distributions -- independent R-MAT matrices, whose rows crowd the low indices --
// every window then holds about u / P entries from the start, where equal row ranges
// overfill the first windows and need several refinement rounds.  Any strictly
// increasing boundaries from 0 to m give the same result; boundary q is forced to
// q + max_{t <= q}(b_t - t) over the candidates b_t clamped to [t, m - P + t], which
// is strictly increasing whatever the rows hold.  Boundary b of column c has index
// wfirst[c] + c + q.
__global__ __launch_bounds__(256) void k_win_fill(PlanParams p, const int* const* __restrict__ cp,
                                                  const int* const* __restrict__ ri, const int* __restrict__ wcols,
                                                  const int* __restrict__ u, int n_wcols,
                                                  const int* __restrict__ wfirst, int* __restrict__ win_c,
                                                  int* __restrict__ brow, int* __restrict__ bcol,
                                                  int* __restrict__ wlin) {
  __shared__ int wl[256 / 64], wi[256 / 64];
  __shared__ int carry_s;
  const int c = blockIdx.x;
  if (c >= n_wcols) return;
  const int w0 = wfirst[c], P = wfirst[c + 1] - w0;
  const int j = wcols[c];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  // the longest input of the column (lowest index among equals)
  int best_len = -1, best_i = 0;
  const bool quant = P > 1 && !p.unsorted_in;
  if (quant) {
    for (int i = threadIdx.x; i < p.k; i += 256) {
      const int* col = cp[i];
      const int len = col[j + 1] - col[j];
      if (len > best_len) {
        best_len = len;
        best_i = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const int ol = __shfl_xor(best_len, off, 64), oi = __shfl_xor(best_i, off, 64);
      if (ol > best_len || (ol == best_len && oi < best_i)) {
        best_len = ol;
        best_i = oi;
      }
    }
    if (lane == 0) {
      wl[w] = best_len;
      wi[w] = best_i;
    }
    __syncthreads();
    best_len = wl[0];
    best_i = wi[0];
    for (int v = 1; v < 256 / 64; ++v)
      if (wl[v] > best_len || (wl[v] == best_len && wi[v] < best_i)) {
        best_len = wl[v];
        best_i = wi[v];
      }
  }
  bool use_q = quant && best_len >= P;
  if (use_q && win_search_linear(u[j], p.k)) {  // (uniform)
    // a column of long runs keeps the equal splits (and the ordered pass) where they
    // hold about equal entries of the longest input: none more than 1.5 times its share
    // s plus the spread of a uniform sample (4 sqrt(s) + 4)
    const int* r0 = ri[best_i] + cp[best_i][j];
    int mx = 0;
    for (int q = threadIdx.x; q < P; q += 256) {
      const int a0 = lower_bound_rows(r0, 0, best_len, (int)(((long long)q * p.m) / P));
      const int a1 = lower_bound_rows(r0, a0, best_len, (int)(((long long)(q + 1) * p.m) / P));
      mx = max(mx, a1 - a0);
    }
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
    __syncthreads();
    if (lane == 0) wl[w] = mx;
    __syncthreads();
    for (int v = 0; v < 256 / 64; ++v) mx = max(mx, wl[v]);
    const double sh = (double)best_len / (double)P;
    if ((double)mx <= 1.5 * sh + 4.0 * sqrt(sh) + 4.0) use_q = false;
  }
  if (wlin && threadIdx.x == 0) wlin[c] = !use_q && !p.unsorted_in && win_search_linear(u[j], p.k) ? 1 : 0;
  const int* rows = use_q ? ri[best_i] + cp[best_i][j] : nullptr;
  if (threadIdx.x == 0) carry_s = INT_MIN;
  __syncthreads();
  for (int base = 0; base <= P; base += 256) {
    const int q = base + threadIdx.x;
    int cand = INT_MIN;  // b_q - q
    if (q <= P) {
      long long b;
      if (!use_q) {
        b = ((long long)q * (long long)p.m) / P;
      } else if (q == 0) {
        b = 0;
      } else if (q == P) {
        b = p.m;
      } else {
        b = rows[(long long)q * best_len / P];
        const long long lo = q, hi = (long long)p.m - P + q;
        b = b < lo ? lo : b > hi ? hi : b;
      }
      cand = (int)(b - q);
    }
    // inclusive prefix max over the block, after the previous chunks' maximum
    int pm = cand;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(pm, off, 64);
      if (lane >= off) pm = max(pm, v);
    }
    __syncthreads();
    if (lane == 63) wl[w] = pm;
    __syncthreads();
    for (int v = 0; v < w; ++v) pm = max(pm, wl[v]);
    pm = max(pm, carry_s);
    if (q <= P) {
      const int b = w0 + c + q;
      brow[b] = q + pm;
      bcol[b] = c;
      if (q < P) win_c[w0 + q] = c;
    }
    __syncthreads();
    if (threadIdx.x == 255) carry_s = pm;
    __syncthreads();
  }
}


// Position of every boundary row in every input column: bpos[b*k + i] = the first
// entry of input i's column at or after boundary row b.
//
// One pass over the window columns' entries instead of a binary search per (boundary,
// input), whose probes fetch a cache line of rows for every four bytes they use.
// Each entry's window is found among the column's boundaries (staged in LDS; searched
// in global memory when there are more), and boundary q's position in input i is the
// first entry of i whose window reaches q: entry e writes the boundaries after its
// predecessor's window (in the same input; none before the input's first entry) up to
// its own, the input's last entry the boundaries after its window up to the column's
// last, with the input's end, and an input with no entry in the column writes all of
// them with its start.  For sorted rows this is the lower bound of every boundary row,
// each written once; for any rows every position lies in the input's column segment
// and every boundary is written.  The positions go first into an input-major copy
// (a column's region holds input i's P + 1 boundaries at i (P + 1) .. i (P + 1) + P),
// so that one input's boundaries share cache lines, and k_win_bpos_t transposes them
// into bpos.
constexpr int WLOC_THREADS = 256;
constexpr int WLOC_EPT = 8;                         // entries per thread per round
constexpr int WLOC_ROUND = WLOC_EPT * WLOC_THREADS;  // a chunk is walked in rounds of this many entries
constexpr int WLOC_LDS = 2048;                      // boundaries of a column staged in LDS

// The window of row r among boundaries b[lo .. hi]: the largest q in [lo, hi) with
// b[q] <= r (lo when none is).
__device__ __forceinline__ int window_of(const int* b, int lo, int hi, int r) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (b[mid] <= r) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One input's segment [s, e) walked by one wavefront (columns with more inputs than the
// segment table): the window is kept as a running maximum along the input.
__device__ __forceinline__ void locate_segment(const int* bnd, int P, const int* __restrict__ r, int s, int e,
                                               int* out) {
  const int lane = lane_id();
  int prevw = -1;  // running window before the chunk (-1 before the first row)
  for (int base = s; base < e; base += 64) {
    const int idx = base + lane;
    const int w = idx < e ? window_of(bnd, 0, P, gload<int>((long long)(r + idx))) : -1;
    const int wm = max(wave_scan_max(w), prevw);
    const int up = __shfl_up(wm, 1, 64);
    const int wprev = lane == 0 ? prevw : up;
    if (idx < e)
      for (int q = wprev + 1; q <= wm; ++q) out[q] = idx;
    prevw = readlane(wm, 63);
  }
  for (int q = prevw + 1 + lane; q <= P; q += 64) out[q] = e;
}

__device__ __forceinline__ void locate_chunk(const PlanParams& p, const int* const* __restrict__ cp,
                                             const int* const* __restrict__ ri, int j, const int* bnd, int P,
                                             int chunk, int nch, const int* segp, const int* segd,
                                             const long long* sega, int* __restrict__ out) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (p.k > WIN_LDS_K) {
    // one chunk per column, one input at a time per wavefront
    for (int i = wv; i < p.k; i += WLOC_THREADS / 64) {
      const int s = cp[i][j], e = cp[i][j + 1];
      locate_segment(bnd, P, ri[i], s, e, out + (long long)i * (P + 1));
    }
    return;
  }
  const int total = segp[p.k];
  int ktop = 0;  // largest power of two <= k - 1
  while ((ktop << 1) <= p.k - 1) ktop = ktop ? ktop << 1 : 1;
  if (p.k == 1) ktop = 0;
  int wtop = 0;  // largest power of two <= P - 1
  while ((wtop << 1) <= P - 1) wtop = wtop ? wtop << 1 : 1;
  if (P <= 1) wtop = 0;
  // this chunk's entries [e0, e_end); the column's last chunk takes every entry after
  // the others (more than its share only where the column totals disagree)
  const bool last = chunk == nch - 1;
  const long long e0l = (long long)chunk * WIN_LOC_CHUNK;
  const int e0 = (int)(e0l < total ? e0l : total);
  const int e_end = last ? total : (int)(e0l + WIN_LOC_CHUNK < total ? e0l + WIN_LOC_CHUNK : total);
  // inputs with no entry in the column: all boundaries at the segment start (written
  // by the chunk holding the segment's place, the last chunk for a trailing one)
  for (int i = tid; i < p.k; i += WLOC_THREADS) {
    const int at = segp[i];
    if (at == segp[i + 1] && ((at >= e0 && at < e_end) || (at == total && last)))
      for (int q = 0; q <= P; ++q) out[(long long)i * (P + 1) + q] = at - segd[i];
  }
  // rounds of WLOC_ROUND entries, wavefront wv taking the WLOC_EPT groups of 64
  // consecutive entries at r0 + 64 (WLOC_EPT wv + t).  The wavefronts need no barrier:
  // the window before a group's first entry is the previous group's last lane, and
  // before the wavefront's first group that of the entry before it, loaded and
  // searched by lane 0.
  const int wbase = wv * 64 * WLOC_EPT;
  for (int r0 = e0; r0 < e_end; r0 += WLOC_ROUND) {  // (uniform)
    const int r1 = e_end - r0 < WLOC_ROUND ? e_end : r0 + WLOC_ROUND;
    const int g0 = r0 + wbase;  // this wavefront's first entry of the round
    if (g0 >= r1) continue;  // (uniform per wavefront; no barrier follows)
    int segv[WLOC_EPT], wv_[WLOC_EPT];
#pragma unroll
    for (int t = 0; t < WLOC_EPT; ++t) segv[t] = 0;
    // the input of each entry: the largest i with segp[i] <= e, all entries' searches
    // step by step (their LDS reads in flight together)
    for (int step = ktop; step > 0; step >>= 1)  // (uniform)
#pragma unroll
      for (int t = 0; t < WLOC_EPT; ++t) {
        const int e = min(g0 + 64 * t + lane, r1 - 1);
        const int c = segv[t] + step;
        if (c < p.k && segp[c] <= e) segv[t] = c;
      }
#pragma unroll
    for (int t = 0; t < WLOC_EPT; ++t) {
      const int e = min(g0 + 64 * t + lane, r1 - 1);  // clamped: no guard on the loads
      wv_[t] = gload<int>(sega[segv[t]] + 4LL * e);
    }
    // lane 0: the entry before the wavefront's first, where that continues its input
    const bool halo = g0 > segp[segv[0]];  // (lane 0's value is the one used)
    int hrow = 0;
    if (lane == 0 && halo) hrow = gload<int>(sega[segv[0]] + 4LL * (g0 - 1));
    // the windows: the largest q < P with bnd[q] <= row, all entries' searches step
    // by step (lane 0 also searches its halo row)
    int lo[WLOC_EPT], hlo = 0;
#pragma unroll
    for (int t = 0; t < WLOC_EPT; ++t) lo[t] = 0;
    for (int step = wtop; step > 0; step >>= 1) {  // (uniform)
#pragma unroll
      for (int t = 0; t < WLOC_EPT; ++t) {
        const int c = lo[t] + step;
        if (c < P && bnd[c] <= wv_[t]) lo[t] = c;
      }
      const int c = hlo + step;
      if (c < P && bnd[c] <= hrow) hlo = c;
    }
#pragma unroll
    for (int t = 0; t < WLOC_EPT; ++t) {
      const int e = g0 + 64 * t + lane;
      const int w = lo[t];
      const int up = __shfl_up(w, 1, 64);
      const int last_prev = t > 0 ? readlane(lo[t > 0 ? t - 1 : 0], 63) : hlo;
      if (e >= r1) continue;
      const int i = segv[t];
      int prev;
      if (e == segp[i]) prev = -1;  // the input's first entry
      else if (lane > 0) prev = up;
      else prev = last_prev;
      const int pos = e - segd[i];  // the entry's position in input i
      int* o = out + (long long)i * (P + 1);
      for (int q = prev + 1; q <= w; ++q) o[q] = pos;
      if (e + 1 == segp[i + 1])  // the input's last entry
        for (int q = w + 1; q <= P; ++q) o[q] = pos + 1;
    }
  }
}

__global__ __launch_bounds__(WLOC_THREADS) void k_win_locate(PlanParams p, const int* const* __restrict__ cp,
                                                             const int* const* __restrict__ ri,
                                                             const int* __restrict__ wcols,
                                                             const int* __restrict__ wfirst,
                                                             const int* __restrict__ brow,
                                                             const int* __restrict__ chfirst,
                                                             const int* __restrict__ chcol, int* __restrict__ bpos_t) {
  // dynamic LDS, sized by the launcher: sega[k] (address of entry e's row: sega[i] + 4 e),
  // segp[k + 1] (exclusive prefix of the segment lengths), segd[k] (segp[i] minus the
  // segment start: entry e is position e - segd[i]); no table past WIN_LDS_K inputs
  extern __shared__ __align__(16) unsigned char smem[];
  const int kt = p.k <= WIN_LDS_K ? p.k : 0;
  long long* sega = reinterpret_cast<long long*>(smem);
  int* segp = reinterpret_cast<int*>(smem + 8 * kt);
  int* segd = segp + kt + 1;
  __shared__ int sb[WLOC_LDS];  // the column's boundary rows
  __shared__ int red[WLOC_THREADS / 64 + 1];
  const int tid = threadIdx.x;
  const int c = chcol[blockIdx.x], chunk = blockIdx.x - chfirst[c];
  const int j = wcols[c];
  const int first = wfirst[c] + c;
  const int P = wfirst[c + 1] - wfirst[c];  // windows; boundaries first .. first + P
  const bool staged = P + 1 <= WLOC_LDS;
  if (staged)
    for (int t = tid; t <= P; t += WLOC_THREADS) sb[t] = brow[first + t];
  if (p.k <= WIN_LDS_K) {
    int carry = 0;
    for (int base = 0; base < p.k; base += WLOC_THREADS) {
      const int i = base + tid;
      int s = 0, len = 0;
      const int* r = nullptr;
      if (i < p.k) {
        r = ri[i];
        s = cp[i][j];
        len = max(cp[i][j + 1] - s, 0);
      }
      int chunk_sum = 0;
      const int ex = block_excl_scan<WLOC_THREADS>(len, red, &chunk_sum);
      if (i < p.k) {
        segp[i] = carry + ex;
        segd[i] = carry + ex - s;
        sega[i] = (long long)(r + s) - 4LL * (carry + ex);
      }
      carry += chunk_sum;
    }
    if (tid == 0) segp[p.k] = carry;
  }
  __syncthreads();
  int* out = bpos_t + (long long)first * p.k;  // the column's region, input-major
  const int nch = chfirst[c + 1] - chfirst[c];
  if (staged) locate_chunk(p, cp, ri, j, sb, P, chunk, nch, segp, segd, sega, out);
  else locate_chunk(p, cp, ri, j, brow + first, P, chunk, nch, segp, segd, sega, out);
}

// bpos[b k + i] from the input-major copy: boundary b = first + q of column c (not
// for the columns of the ordered pass, which writes bpos itself).
__global__ __launch_bounds__(256) void k_win_bpos_t(long long total, int k, const int* __restrict__ bcol,
                                                    const int* __restrict__ wfirst, const int* __restrict__ wlin,
                                                    const int* __restrict__ bpos_t, int* __restrict__ bpos) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const int b = (int)(t / k), i = (int)(t - (long long)b * k);
  const int c = bcol[b];
  if (wlin[c]) return;
  const int first = wfirst[c] + c, P = wfirst[c + 1] - wfirst[c];
  bpos[t] = bpos_t[(long long)first * k + (long long)i * (P + 1) + (b - first)];
}

// The ordered pass: block (c, g) takes inputs 16 g .. 16 g + 15 of window column c, a
// wavefront one input at a time.  The boundaries are the equal row splits
// B_q = floor(q m / P), so a row's window is arithmetic: the largest q < P with
// q m <= (row + 1) P - 1 (a floating-point estimate, corrected by exact integer
// compares).  Along an input the window index of its rows is kept as a running
// maximum (so it never decreases, whatever the input), and boundary q's position is
// the first row whose window reaches q; boundaries after the last row's window are at
// the segment end.  Every boundary of the input is written once.
constexpr int WSL_THREADS = 256;
constexpr int WSL_GROUP = 16;
__global__ __launch_bounds__(WSL_THREADS) void k_win_search_lin(PlanParams p, const int* const* __restrict__ cp,
                                                                const int* const* __restrict__ ri,
                                                                const int* __restrict__ wcols,
                                                                const int* __restrict__ wfirst,
                                                                const int* __restrict__ wlin,
                                                                int* __restrict__ bpos) {
  const int groups = (p.k + WSL_GROUP - 1) / WSL_GROUP;
  const int c = blockIdx.x / groups, g = blockIdx.x - c * groups;
  if (!wlin[c]) return;  // k_win_locate's column
  const int j = wcols[c];
  const int first = wfirst[c] + c;
  const int P = wfirst[c + 1] - wfirst[c];
  const long long k = p.k, m = p.m;
  const double inv_m = 1.0 / (double)m;
  const int lane = lane_id();
  const int i1 = min(p.k, (g + 1) * WSL_GROUP);
  for (int i = g * WSL_GROUP + (threadIdx.x >> 6); i < i1; i += WSL_THREADS / 64) {
    const int* col = cp[i];
    const int s = col[j], e = col[j + 1];
    const int* r = ri[i];
    int* out = bpos + (long long)first * k + i;  // boundary q at out[q * k]
    if (lane == 0) {
      out[0] = s;
      out[(long long)P * k] = e;
    }
    int prevw = 0;  // window of the row before the chunk (0 before the first row)
    for (int base = s; base < e; base += 64) {
      const int idx = base + lane;
      int w = -1;
      if (idx < e) {
        const long long lim = ((long long)gload<int>((long long)(r + idx)) + 1) * P - 1;
        long long q = (long long)((double)lim * inv_m);
        q = q < 0 ? 0 : q > P - 1 ? P - 1 : q;
        while (q > 0 && q * m > lim) --q;
        while (q < P - 1 && (q + 1) * m <= lim) ++q;
        w = (int)q;
      }
      const int wm = max(wave_scan_max(w), prevw);
      const int up = __shfl_up(wm, 1, 64);
      const int wprev = lane == 0 ? prevw : up;
      if (idx < e)
        for (int q = wprev + 1; q <= wm; ++q) out[(long long)q * k] = idx;
      prevw = readlane(wm, 63);
    }
    for (int q = prevw + 1 + lane; q <= P - 1; q += 64) out[(long long)q * k] = e;
  }
}

// Input count of every window; windows with more than cap_in entries and more than
// cap_in rows are cut into q equal row ranges (q[w] = 1 otherwise).  One wavefront
// per window at a time, lane i reading input i's two boundary positions (coalesced:
// the k positions of a boundary are contiguous), windows dealt out over the launch's
// wavefronts.
__global__ __launch_bounds__(256) void k_win_count(PlanParams p, int n_windows, const int* __restrict__ win_c,
                                                   const int* __restrict__ brow, const int* __restrict__ bpos,
                                                   int* __restrict__ cntin, int* __restrict__ q,
                                                   PlanSummary* __restrict__ sum) {
  const int lane = lane_id();
  const int nwave = (int)gridDim.x * 4;
  int wmax = 0, nref = 0;  // over this wavefront's windows
  for (int w = blockIdx.x * 4 + (threadIdx.x >> 6); w < n_windows; w += nwave) {
    const int b = w + win_c[w];
    long long cnt = 0;
    if (bpos) {
      const int* lo = bpos + (long long)b * p.k;
      const int* hi = lo + p.k;
      long long part = 0;
      for (int i = lane; i < p.k; i += 64) part += max(hi[i] - lo[i], 0);  // (inverted only for an unsorted input)
      cnt = wave_sum<long long>(part);
    } else {
      cnt = cntin[w];  // counted by histogram (unsorted input)
    }
    const int width = brow[b + 1] - brow[b];
    wmax = max(wmax, width);
    int pieces = 1;
    long long qq = 1;
    if (cnt > p.cap_in && width > p.cap_in) {
      const double target = (double)p.cap_in * (double)p.win_fill;
      qq = (long long)ceil((double)cnt / (target > 1.0 ? target : 1.0));
      if (qq < 2) qq = 2;
    }
    if (width > p.win_span) {  // wider than the workgroup bitmap: equal pieces that fit it
      const long long qw = ((long long)width + p.win_span - 1) / p.win_span;
      if (qw > qq) qq = qw;
    }
    if (qq > 1) {
      if (qq > width) qq = width;
      pieces = (int)qq;
      ++nref;
    }
    if (lane == 0) {
      cntin[w] = cnt > INT_MAX ? INT_MAX : (int)cnt;
      q[w] = pieces;
    }
  }
  // the widest window and the windows still to refine: one atomic of each per
  // wavefront (one per window would all go to the same two words)
  if (lane == 0) {
    if (wmax > 0) atomicMax(&sum->max_span, wmax);
    if (nref) atomicAdd(&sum->pad, nref);
  }
}

// One refinement level: window w becomes q[w] row ranges.  newfirst is the exclusive
// scan of q.  With the boundary positions of sorted inputs (bpos_old) a window no wider
// than the workgroup bitmap is cut at row quantiles of its longest input within the
// window (as the first windows are, so the pieces hold about equal entries and one
// level mostly suffices on skewed rows); otherwise, and for a window cut for its
// width, into equal row ranges.  The cuts are forced strictly increasing inside the
// window, so any rows give valid windows.
__global__ __launch_bounds__(256) void k_win_refine_fill(int n_windows, int n_wcols, const int* __restrict__ win_c,
                                                         const int* __restrict__ wfirst_old,
                                                         const int* __restrict__ q,
                                                         const int* __restrict__ newfirst,
                                                         const int* __restrict__ brow_old, int k, int win_span,
                                                         const int* const* __restrict__ ri,
                                                         const int* __restrict__ bpos_old,
                                                         int* __restrict__ win_c_new, int* __restrict__ brow_new,
                                                         int* __restrict__ bcol_new, int* __restrict__ bpar,
                                                         int* __restrict__ bpiece, int* __restrict__ wfirst_new) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w < n_windows) {
    const int c = win_c[w];
    const int pieces = q[w], nw0 = newfirst[w];
    const int rlo = brow_old[w + c], rhi = brow_old[w + c + 1];
    // the window's longest input (lowest index among equals)
    int best_len = 0, best_lo = 0, best_i = 0;
    if (bpos_old && pieces > 1 && rhi - rlo <= win_span) {
      const int* lo = bpos_old + (long long)(w + c) * k;
      const int* hi = lo + k;
      for (int i = 0; i < k; ++i) {
        const int len = hi[i] - lo[i];
        if (len > best_len) {
          best_len = len;
          best_lo = lo[i];
          best_i = i;
        }
      }
    }
    const bool quant = best_len >= pieces;
    const int* rows = quant ? ri[best_i] : nullptr;
    int prev = rlo;
    for (int t = 0; t < pieces; ++t) {
      const int nb = nw0 + t + c;
      int b;
      if (t == 0) {
        b = rlo;
      } else if (quant) {
        b = rows[best_lo + (int)(((long long)t * best_len) / pieces)];
        b = max(b, prev + 1);
        b = min(b, rhi - (pieces - t));
      } else {
        b = rlo + (int)(((long long)t * (long long)(rhi - rlo)) / pieces);
      }
      prev = b;
      brow_new[nb] = b;
      bcol_new[nb] = c;
      bpar[nb] = w;
      bpiece[nb] = t;
      win_c_new[nw0 + t] = c;
    }
    if (w + 1 == wfirst_old[c + 1]) {  // last window of its column: also the end boundary
      const int nb = nw0 + pieces + c;
      brow_new[nb] = rhi;
      bcol_new[nb] = c;
      bpar[nb] = w;
      bpiece[nb] = pieces;
    }
  }
  if (w <= n_wcols) wfirst_new[w] = newfirst[wfirst_old[w]];
}

__global__ __launch_bounds__(256) void k_win_refine_search(PlanParams p, const int* const* __restrict__ ri,
                                                           int n_bounds_new, const int* __restrict__ bcol_new,
                                                           const int* __restrict__ brow_new,
                                                           const int* __restrict__ bpar,
                                                           const int* __restrict__ bpiece,
                                                           const int* __restrict__ q,
                                                           const int* __restrict__ bpos_old,
                                                           int* __restrict__ bpos_new) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)n_bounds_new * p.k) return;
  const int nb = (int)(t / p.k), i = (int)(t - (long long)nb * p.k);
  const int w = bpar[nb], piece = bpiece[nb], c = bcol_new[nb];
  const int ob = w + c;  // old lower boundary of the parent window
  const int lo = bpos_old[(long long)ob * p.k + i], hi = bpos_old[(long long)(ob + 1) * p.k + i];
  int pos;
  if (piece == 0) pos = lo;
  else if (piece == q[w]) pos = hi;
  else pos = lower_bound_rows(ri[i], lo, hi, brow_new[nb]);
  bpos_new[t] = pos;
}

// The final windows as one record each (column id, rows [rlo, rhi), lower boundary):
// a window kernel then starts from one load instead of a chain of three.
__global__ __launch_bounds__(256) void k_win_records(int n_windows, const int* __restrict__ wcols,
                                                     const int* __restrict__ win_c, const int* __restrict__ brow,
                                                     int4* __restrict__ wrec) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= n_windows) return;
  const int c = win_c[w];
  const int b = w + c;
  wrec[w] = make_int4(wcols[c], brow[b], brow[b + 1], b);
}

// Per window column: nnz(B(:,j)) = sum of its window counts, and each window's
// offset inside the column.
__global__ __launch_bounds__(256) void k_win_colsum(int n_wcols, const int* __restrict__ wcols,
                                                    const int* __restrict__ wfirst,
                                                    const int* __restrict__ win_cnt, int* __restrict__ colcnt,
                                                    int* __restrict__ win_off) {
  __shared__ int scratch[256 / 64 + 1];
  const int c = blockIdx.x;
  if (c >= n_wcols) return;
  const int w0 = wfirst[c], w1 = wfirst[c + 1];
  int carry = 0;
  for (int base = w0; base < w1; base += 256) {
    const int w = base + threadIdx.x;
    const int v = w < w1 ? win_cnt[w] : 0;
    int chunk = 0;
    const int ex = block_excl_scan<256>(v, scratch, &chunk);
    if (w < w1) win_off[w] = carry + ex;
    carry += chunk;
  }
  if (threadIdx.x == 0) colcnt[wcols[c]] = carry;
}

// ---- exclusive scan of int32 counts: tile sums, then each tile adds the sums of
// the tiles before it (two kernels, no single-block pass) ----
constexpr int SCAN_THREADS = 256, SCAN_PER_THREAD = 16, SCAN_TILE = SCAN_THREADS * SCAN_PER_THREAD;

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const int* __restrict__ in, long long len,
                                                              long long* __restrict__ bsum) {
  __shared__ long long scratch[SCAN_THREADS / 64 + 1];
  const long long base = (long long)blockIdx.x * SCAN_TILE;
  const int tlen = (int)(len - base < SCAN_TILE ? len - base : SCAN_TILE);  // >= 1
  long long s = 0;
#pragma unroll
  for (int t = 0; t < SCAN_PER_THREAD; ++t) {
    const int x = t * SCAN_THREADS + (int)threadIdx.x;
    const int v = in[base + min(x, tlen - 1)];  // clamped index: no guard on the load
    s += x < tlen ? v : 0;
  }
  s = block_sum<SCAN_THREADS>(s, scratch);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

// Long inputs: exclusive scan of the tile sums in place, total into bsum[nb].
__global__ __launch_bounds__(1024) void k_scan_top(long long* __restrict__ bsum, int nb) {
  __shared__ long long scratch[1024 / 64 + 1];
  long long carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int t = base + threadIdx.x;
    const long long v = t < nb ? bsum[t] : 0;
    long long chunk = 0;
    const long long ex = block_excl_scan<1024>(v, scratch, &chunk);
    if (t < nb) bsum[t] = carry + ex;
    carry += chunk;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

// Block b: prefix = sum of bsum[0..b) and total = sum of bsum[0..nb), summed here
// (short inputs) or read from k_scan_top's output (prefixed).  Block 0 also writes
// out[len] and the total.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const int* __restrict__ in, long long len,
                                                             const long long* __restrict__ bsum, int nb,
                                                             bool prefixed, long long* __restrict__ total,
                                                             int* __restrict__ out, int* __restrict__ err) {
  __shared__ long long scratch[SCAN_THREADS / 64 + 1];
  long long pre = 0, all = 0;
  if (prefixed) {
    pre = bsum[blockIdx.x];
    all = bsum[nb];
  } else {
    for (int t = threadIdx.x; t < nb; t += SCAN_THREADS) {
      const long long v = bsum[t];
      pre += t < (int)blockIdx.x ? v : 0;
      all += v;
    }
    pre = block_sum<SCAN_THREADS>(pre, scratch);
    all = block_sum<SCAN_THREADS>(all, scratch);
  }
  if (all > INT_MAX) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *total = all;
      atomicOr(err, ERR_OVERFLOW);
    }
    return;
  }
  // the tile through LDS: coalesced loads and stores, SCAN_PER_THREAD consecutive
  // entries scanned per thread
  __shared__ int buf[SCAN_TILE];
  const long long tile = (long long)blockIdx.x * SCAN_TILE;
  const int tlen = (int)(len - tile < SCAN_TILE ? len - tile : SCAN_TILE);
  if (tlen <= 0) return;  // (uniform; the launcher sends only len > SCAN_SMALL here)
#pragma unroll
  for (int q = 0; q < SCAN_PER_THREAD; ++q) {
    const int x = q * SCAN_THREADS + (int)threadIdx.x;
    const int v = in[tile + min(x, tlen - 1)];  // clamped index: no guard on the load
    buf[x] = x < tlen ? v : 0;
  }
  __syncthreads();
  int v[SCAN_PER_THREAD];
  long long s = 0;
#pragma unroll
  for (int t = 0; t < SCAN_PER_THREAD; ++t) {
    v[t] = buf[threadIdx.x * SCAN_PER_THREAD + t];
    s += v[t];
  }
  long long run = pre + block_excl_scan<SCAN_THREADS>(s, scratch);
#pragma unroll
  for (int t = 0; t < SCAN_PER_THREAD; ++t) {
    buf[threadIdx.x * SCAN_PER_THREAD + t] = (int)run;
    run += v[t];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < SCAN_PER_THREAD; ++q) {
    const int x = q * SCAN_THREADS + (int)threadIdx.x;
    if (x < tlen) out[tile + x] = buf[x];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[len] = (int)all;
    *total = all;
  }
}

// Short inputs (len <= SCAN_SMALL): the whole scan in one workgroup, one launch.
constexpr int SCAN_SMALL_THREADS = 1024, SCAN_SMALL_PER = 16;
constexpr long long SCAN_SMALL = SCAN_SMALL_THREADS * SCAN_SMALL_PER;  // one tile, 16384
__global__ __launch_bounds__(SCAN_SMALL_THREADS) void k_scan_small(const int* __restrict__ in, int len,
                                                                   long long* __restrict__ total,
                                                                   int* __restrict__ out, int* __restrict__ err) {
  __shared__ long long scratch[SCAN_SMALL_THREADS / 64 + 1];
  __shared__ int buf[SCAN_SMALL_THREADS * SCAN_SMALL_PER];
  const long long all = block_scan_counts<SCAN_SMALL_THREADS, SCAN_SMALL_PER>(in, len, out, scratch, buf);
  if (threadIdx.x == 0) {
    *total = all;
    if (all > INT_MAX) atomicOr(err, ERR_OVERFLOW);
    else out[len] = (int)all;
  }
}

// ---- host launchers ----
static inline unsigned grid_for(long long work, int per_block) {
  return (unsigned)((work + per_block - 1) / per_block);
}

void launch_bounds(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, int* d_u,
                   unsigned char* d_bin, int* d_colcnt, int* d_hist, PlanSummary* d_sum, hipStream_t s) {
  const unsigned grid = p.n == 0 ? 1u : grid_for(p.n, PLAN_THREADS);
  k_bounds<<<grid, PLAN_THREADS, 0, s>>>(p, d_cp, d_ri, d_u, d_bin, d_colcnt, d_hist, d_sum);
}

void launch_put_ptrs(const void* const* host_ptrs, int count, const void** d_dst, PlanSummary* d_sum,
                     void* d_dummy, hipStream_t s) {
  for (int base = 0; base < count || base == 0; base += PtrChunk::kMax) {
    PtrChunk c;
    c.count = count - base < PtrChunk::kMax ? count - base : PtrChunk::kMax;
    for (int i = 0; i < c.count; ++i) c.p[i] = host_ptrs[base + i];
    k_put_ptrs<<<1, 256, 0, s>>>(c, d_dst + base, base == 0 ? d_sum : nullptr,
                                 base == 0 ? (unsigned*)d_dummy : nullptr);
    if (count <= 0) break;
  }
}

void launch_validate(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, PlanSummary* d_sum,
                     hipStream_t s) {
  if (p.n == 0) return;
  k_validate<<<grid_for(p.n, PLAN_THREADS), PLAN_THREADS, 0, s>>>(p, d_cp, d_ri, d_sum);
}

void launch_bin_scan(int nblk, bool merge, int* d_hist, int* d_binoff, PlanSummary* d_sum, hipStream_t s) {
  k_bin_scan<<<1, 1024, 0, s>>>(nblk, merge ? 1 : 0, d_hist, d_binoff, d_sum);
}

void launch_bin_scatter(const PlanParams& p, const unsigned char* d_bin, const int* d_hist, const int* d_binoff,
                        int* d_list, hipStream_t s) {
  if (p.n == 0) return;
  k_bin_scatter<<<grid_for(p.n, PLAN_THREADS), PLAN_THREADS, 0, s>>>(p, d_bin, d_hist, d_binoff, d_list);
}

void launch_win_scan(const PlanParams& p, const int* d_list, const int* d_binoff, const int* d_u, int* d_wfirst,
                     PlanSummary* d_sum, hipStream_t s) {
  k_win_scan<<<1, 1024, 0, s>>>(p, d_list, d_binoff, d_u, d_wfirst, d_sum);
}

void launch_win_fill(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, const int* d_wcols,
                     const int* d_u, int n_wcols, const int* d_wfirst, int* d_win_c, int* d_brow, int* d_bcol,
                     int* d_wlin, hipStream_t s) {
  if (n_wcols == 0) return;
  k_win_fill<<<n_wcols, 256, 0, s>>>(p, d_cp, d_ri, d_wcols, d_u, n_wcols, d_wfirst, d_win_c, d_brow, d_bcol,
                                     d_wlin);
}

void launch_win_search(const PlanParams& p, const int* const* d_cp, const int* const* d_ri, const int* d_wcols,
                       const int* d_wfirst, const int* d_wlin, int n_wcols, const int* d_brow, const int* d_bcol,
                       int n_bounds, int n_chunks, const int* d_chfirst, const int* d_chcol, int* d_bpos_t,
                       int* d_bpos, hipStream_t s) {
  if (n_wcols <= 0 || p.k == 0) return;
  const long long groups = (p.k + WSL_GROUP - 1) / WSL_GROUP;
  k_win_search_lin<<<(unsigned)(n_wcols * groups), WSL_THREADS, 0, s>>>(p, d_cp, d_ri, d_wcols, d_wfirst, d_wlin,
                                                                         d_bpos);
  if (n_chunks <= 0) return;
  const int kt = p.k <= WIN_LDS_K ? p.k : 0;
  const size_t lds = (size_t)8 * kt + 4 * (2 * (size_t)kt + 1);
  k_win_locate<<<(unsigned)n_chunks, WLOC_THREADS, lds, s>>>(p, d_cp, d_ri, d_wcols, d_wfirst, d_brow, d_chfirst,
                                                            d_chcol, d_bpos_t);
  const long long total = (long long)n_bounds * p.k;
  k_win_bpos_t<<<grid_for(total, 256), 256, 0, s>>>(total, p.k, d_bcol, d_wfirst, d_wlin, d_bpos_t, d_bpos);
}

void launch_win_count(const PlanParams& p, int n_windows, const int* d_win_c, const int* d_brow, const int* d_bpos,
                      int* d_cntin, int* d_q, PlanSummary* d_sum, hipStream_t s) {
  if (n_windows == 0) return;
  // one wavefront per window at a time: about 16 windows per wavefront
  const int blocks = (int)((n_windows + 63) / 64) > 4096 ? 4096 : (int)((n_windows + 63) / 64);
  k_win_count<<<blocks > 0 ? blocks : 1, 256, 0, s>>>(p, n_windows, d_win_c, d_brow, d_bpos, d_cntin, d_q, d_sum);
}

void launch_win_refine_fill(const PlanParams& p, int n_windows, int n_wcols, const int* d_win_c,
                            const int* d_wfirst_old, const int* d_q, const int* d_newfirst, const int* d_brow_old,
                            const int* const* d_ri, const int* d_bpos_old, int* d_win_c_new, int* d_brow_new,
                            int* d_bcol_new, int* d_bpar, int* d_bpiece, int* d_wfirst_new, hipStream_t s) {
  const int work = (n_windows > n_wcols + 1 ? n_windows : n_wcols + 1);
  k_win_refine_fill<<<grid_for(work, 256), 256, 0, s>>>(n_windows, n_wcols, d_win_c, d_wfirst_old, d_q,
                                                        d_newfirst, d_brow_old, p.k, p.win_span, d_ri, d_bpos_old,
                                                        d_win_c_new, d_brow_new, d_bcol_new, d_bpar, d_bpiece,
                                                        d_wfirst_new);
}

void launch_win_refine_search(const PlanParams& p, const int* const* d_ri, int n_bounds_new, const int* d_bcol_new,
                              const int* d_brow_new, const int* d_bpar, const int* d_bpiece, const int* d_q,
                              const int* d_bpos_old, int* d_bpos_new, hipStream_t s) {
  const long long work = (long long)n_bounds_new * p.k;
  if (work == 0) return;
  k_win_refine_search<<<grid_for(work, 256), 256, 0, s>>>(p, d_ri, n_bounds_new, d_bcol_new, d_brow_new, d_bpar,
                                                          d_bpiece, d_q, d_bpos_old, d_bpos_new);
}

void launch_win_records(int n_windows, const int* d_wcols, const int* d_win_c, const int* d_brow, int4* d_wrec,
                        hipStream_t s) {
  if (n_windows <= 0) return;
  k_win_records<<<grid_for(n_windows, 256), 256, 0, s>>>(n_windows, d_wcols, d_win_c, d_brow, d_wrec);
}

void launch_win_colsum(int n_wcols, const int* d_wcols, const int* d_wfirst, const int* d_win_cnt, int* d_colcnt,
                       int* d_win_off, hipStream_t s) {
  if (n_wcols == 0) return;
  k_win_colsum<<<n_wcols, 256, 0, s>>>(n_wcols, d_wcols, d_wfirst, d_win_cnt, d_colcnt, d_win_off);
}

size_t scan_tmp_bytes(int64_t len) {
  const int64_t nb = (len + SCAN_TILE - 1) / SCAN_TILE;
  return (size_t)(nb + 1) * sizeof(long long);
}

void launch_scan(const int* d_in, int64_t len, int* d_out, long long* d_total, int* d_err, void* d_tmp,
                 hipStream_t s) {
  // one workgroup for one tile; longer inputs in parallel tiles (measured: one
  // workgroup walking the four tiles of 65536 counts takes 18 us, the two launches
  // below 10 us)
  if (len <= SCAN_SMALL) {
    k_scan_small<<<1, SCAN_SMALL_THREADS, 0, s>>>(d_in, (int)len, d_total, d_out, d_err);
    return;
  }
  const int nb = (int)((len + SCAN_TILE - 1) / SCAN_TILE);
  long long* bsum = (long long*)d_tmp;
  if (nb > 0) k_scan_reduce<<<nb, SCAN_THREADS, 0, s>>>(d_in, len, bsum);
  const bool prefixed = nb > 1024;
  if (prefixed) k_scan_top<<<1, 1024, 0, s>>>(bsum, nb);
  k_scan_apply<<<nb > 0 ? nb : 1, SCAN_THREADS, 0, s>>>(d_in, len, bsum, nb, prefixed, d_total, d_out, d_err);
}

}  // namespace spk
