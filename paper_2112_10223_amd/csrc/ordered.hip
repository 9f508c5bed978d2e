// Ordered values (SPKADD_FLAG_ORDERED).
//
// Algorithm 5 visits the inputs of a column in order i = 1..k and adds each entry
// into the slot of its row, so each output value is the sequential sum of its terms
// in input order.  The numeric kernels add in the order their atomics happen to
// meet, which is bounded by the summation error bound but not reproducible bit for
// bit.  This pass runs after the numeric pass has written the sorted rows of B and
// sums every output entry again in input order, one rounding per addition in the
// values' own type: the first term is stored, each later term added.
//
// One wavefront per unit (a column, or a row window of a window column).  The unit's
// output rows go to LDS with a "touched" byte per slot.  The unit's input entries are
// numbered input by input (input i's entries before input i+1's, each input in its
// stored order) and taken 64 at a time; an entry's output slot is found by a binary
// search over the unit's sorted rows.  Within a group of 64 the lanes are applied
// one input at a time, so a slot receives its terms in input order; rows are unique
// within an input column, so the lanes of one input never share a slot.  One
// wavefront's LDS accesses complete in program order.
#include <climits>

#include "device.h"
#include "internal.h"
#include "ordered.h"

namespace spk {

namespace {

constexpr int ORD_THREADS = 64;

// LDS layout of one unit (bytes): base addresses of the k inputs' rows and values
// (shifted so that the unit's entry number addresses them), k + 1 segment starts,
// then the output rows, values and touched bytes of up to cap slots.
struct OrdLayout {
  int off_rb, off_vb, off_ss, off_rows, off_vals, off_touch, bytes;
};

__host__ __device__ inline OrdLayout ord_layout(int k, int cap, int vbytes) {
  OrdLayout L;
  int off = 0;
  L.off_rb = off;
  off += 8 * k;
  L.off_vb = off;
  off += 8 * k;
  L.off_ss = off;
  off += 4 * (k + 1);
  off = (off + 15) & ~15;
  L.off_rows = off;
  off += 4 * cap;
  off = (off + 15) & ~15;
  L.off_vals = off;
  off += vbytes * cap;
  L.off_touch = off;
  off += cap;
  L.bytes = (off + 15) & ~15;
  return L;
}

// Units [0, ncols) are the listed columns, units [ncols, ncols + nwin) the row windows.
template <typename V>
__global__ __launch_bounds__(ORD_THREADS) void k_ordered(KArgs a, const int* __restrict__ cols, int ncols, int nwin,
                                                         int cap) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int k = a.k;
  const OrdLayout L = ord_layout(k, cap, (int)sizeof(V));
  long long* rb = reinterpret_cast<long long*>(lds + L.off_rb);
  long long* vb = reinterpret_cast<long long*>(lds + L.off_vb);
  int* ss = reinterpret_cast<int*>(lds + L.off_ss);
  int* orow = reinterpret_cast<int*>(lds + L.off_rows);
  V* oval = reinterpret_cast<V*>(lds + L.off_vals);
  unsigned char* touched = lds + L.off_touch;
  const int lane = lane_id();
  const int total = ncols + nwin;
  for (int unit = blockIdx.x; unit < total; unit += gridDim.x) {
    const bool win = unit >= ncols;
    int j, o0, c, b = 0;
    if (!win) {
      j = cols[unit];
      o0 = a.colptr_c[j];
      c = a.colptr_c[j + 1] - o0;
    } else {
      const int w = unit - ncols;
      const int4 rec = a.wrec[w];
      j = rec.x;
      b = rec.w;
      o0 = a.colptr_c[j] + a.win_off[w];
      c = a.win_cnt[w];
    }
    if (c > cap) {  // (cannot happen for a plan's own units)
      if (lane == 0) atomicOr(a.err, ERR_COUNT);
      continue;
    }
    // segment table: input i's entries of the unit are numbers [ss[i], ss[i+1])
    int carry = 0;
    for (int i0 = 0; i0 < k; i0 += 64) {
      const int i = i0 + lane;
      int s = 0, e = 0;
      if (i < k) {
        if (!win) {
          const int* cp = a.cp[i];
          s = cp[j];
          e = cp[j + 1];
        } else {
          s = a.bpos[(long long)b * k + i];
          e = a.bpos[(long long)(b + 1) * k + i];
        }
        if (e < s) e = s;
      }
      const int len = e - s;
      const int incl = wave_scan_add(len);
      const int ex = carry + incl - len;
      if (i < k) {
        ss[i] = ex;
        rb[i] = (long long)(a.ri[i] + s) - 4LL * ex;
        vb[i] = (long long)((const V*)a.va[i] + s) - (long long)sizeof(V) * ex;
      }
      carry += readlane(incl, 63);
    }
    if (lane == 0) ss[k] = carry;
    const int u = carry;
    for (int q = lane; q < c; q += 64) {
      orow[q] = a.out_r[o0 + q];
      touched[q] = 0;
    }
    wave_sync();
    for (int base = 0; base < u; base += 64) {
      const int p = base + lane;
      const bool in = p < u;
      const int pp = in ? p : u - 1;
      // the input of entry pp: the last i with ss[i] <= pp (its segment is non-empty)
      int lo = 0, hi = k - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ss[mid] <= pp) lo = mid;
        else hi = mid - 1;
      }
      const int seg = lo;
      const int row = gload<int>(rb[seg] + 4LL * pp);
      const V val = gload<V>(vb[seg] + (long long)sizeof(V) * pp);
      int l2 = 0, h2 = c;
      while (l2 < h2) {
        const int mid = (l2 + h2) >> 1;
        if (orow[mid] < row) l2 = mid + 1;
        else h2 = mid;
      }
      const bool found = l2 < c && orow[l2] == row;
      if (in && !found) atomicOr(a.err, ERR_COUNT);
      const int s_lo = readlane(seg, 0);
      const int s_hi = readlane(seg, min(63, u - 1 - base));
      for (int sg = s_lo; sg <= s_hi; ++sg) {
        if (in && found && seg == sg) {
          if (touched[l2]) {
            oval[l2] = oval[l2] + val;
          } else {
            oval[l2] = val;
            touched[l2] = 1;
          }
        }
        wave_sync();
      }
    }
    for (int q = lane; q < c; q += 64) {
      if (!touched[q]) atomicOr(a.err, ERR_COUNT);
      gstore<V>((long long)((V*)a.out_v + o0 + q), oval[q]);
    }
    wave_sync();
  }
}

}  // namespace

int ordered_lds_bytes(int k, int cap, int vbytes) { return ord_layout(k, cap, vbytes).bytes; }

hipError_t launch_ordered(const KArgs& a, const int* d_cols, int ncols, int nwin, int cap, bool f64, int n_cu,
                          hipStream_t s) {
  const int total = ncols + nwin;
  if (total <= 0) return hipSuccess;
  const size_t lds = (size_t)ordered_lds_bytes(a.k, cap, f64 ? 8 : 4);
  long long per_cu = (long long)max_lds_bytes() / (long long)(lds > 0 ? lds : 1);
  if (per_cu > 32) per_cu = 32;
  if (per_cu < 1) per_cu = 1;
  long long grid = per_cu * n_cu;
  if (grid > total) grid = total;
  if (f64)
    k_ordered<double><<<(int)grid, ORD_THREADS, lds, s>>>(a, d_cols, ncols, nwin, cap);
  else
    k_ordered<float><<<(int)grid, ORD_THREADS, lds, s>>>(a, d_cols, ncols, nwin, cap);
  return hipGetLastError();
}

}  // namespace spk
