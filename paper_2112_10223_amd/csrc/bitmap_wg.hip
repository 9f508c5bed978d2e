// Workgroup bitmap accumulator for row windows (Section III-B, Algorithms 7-8) and
// workgroup columns whose row range is narrow enough: one bit per row of the unit's
// range [rlo, rhi) in LDS.  Symbolic (Algorithm 6): an OR that finds its bit clear
// counts a new row.  Numeric (Algorithm 5): OR with return marks each row's first
// entry, a block-wide popcount prefix over word pairs gives rank(row) = the row's
// position in the sorted output, the first entry stores (row, value) at its rank in
// an LDS staging area and later entries add by compare-and-swap; the unit is then
// written out coalesced.  No hash table and no sort: the bitmap is the "partitioned
// SPA" the paper proposes for row-partitioned accumulation, with a rank in place of a
// dense value array.
//
// A unit wider than a.wg_span_max rows is left to the hash kernel (k_hash_wg skips the
// units this kernel takes, so both can run over one unit list).
#include "wave_device.h"

namespace spk {

template <int NT, int EW, bool NUM, bool WIN, typename V>
__global__ __launch_bounds__(NT) void k_bitmap_wg(KArgs a, const int* __restrict__ list, int nunits) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long red[NT / 64 + 1];
  __shared__ int info;
  const int unit = xcd_remap(blockIdx.x, gridDim.x);
  if (unit >= nunits) return;  // uniform over the block
  const int tid = threadIdx.x;
  int j, blo = 0, rlo = 0, rhi = a.m;
  if (WIN) {
    const int c = a.win_c[unit];
    j = a.wcols[c];
    blo = unit + c;
    rlo = a.brow[blo];
    rhi = a.brow[blo + 1];
  } else {
    j = list[unit];
  }
  const int span = rhi - rlo;
  if (span > a.wg_span_max) return;  // the hash kernel's unit (uniform)
  unsigned* bm = reinterpret_cast<unsigned*>(smem);
  unsigned short* pw = reinterpret_cast<unsigned short*>(smem + a.off_pre);  // set bits below each word pair
  int* P = reinterpret_cast<int*>(smem + a.off_P);
  long long* adj = reinterpret_cast<long long*>(smem + a.off_adj);
  long long* adjv = reinterpret_cast<long long*>(smem + a.off_adjv);
  if (tid < 64) {
    const int u = build_meta<NUM, V>(a, j, WIN, blo, P, adj, adjv);
    if (tid == 0) info = u;
  }
  const int npair = (span + 63) >> 6;
  for (int w = tid; w < 2 * npair; w += NT) bm[w] = 0u;
  __syncthreads();
  const int u = info;
  const bool one = u <= NT * EW;  // every entry of the unit in registers at once
  int rows[EW];
  V vals[EW];
  bool first[EW];
  int newc = 0, bad = 0;
  for (int cb = 0; cb < u; cb += NT * EW) {
#pragma unroll
    for (int t = 0; t < EW; ++t) {
      const int e = cb + tid + NT * t;
      rows[t] = rlo;
      if (e < u) {
        const int sg = seg_of(P, a.k, a.ktop, e);
        rows[t] = gload<int>(adj[sg] + 4LL * e);
        if (NUM && one) vals[t] = gload<V>(adjv[sg] + (long long)sizeof(V) * e);
      }
    }
#pragma unroll
    for (int t = 0; t < EW; ++t) {
      const int e = cb + tid + NT * t;
      const int r = rows[t] - rlo;
      const bool in = e < u && (unsigned)r < (unsigned)span;
      bad |= e < u && !in;  // a row outside the unit's range: invalid input
      const unsigned bit = in ? 1u << (r & 31) : 0u;
      const unsigned old = in ? atomicOr(&bm[r >> 5], bit) : bit;
      first[t] = in && (old & bit) == 0u;
      newc += first[t] ? 1 : 0;
    }
  }
  if (bad) atomicOr(a.err, ERR_INPUT);
  __syncthreads();
  if (!NUM) {
    const long long total = block_sum<NT, long long>((long long)newc, red);
    if (tid == 0) {
      if (WIN) a.win_cnt[unit] = (int)total;
      else a.colcnt[j] = (int)total;
    }
    return;
  }
  int cnt, o0;
  if (WIN) {
    cnt = a.win_cnt[unit];
    o0 = a.colptr_c[j] + a.win_off[unit];
  } else {
    o0 = a.colptr_c[j];
    cnt = a.colptr_c[j + 1] - o0;
  }
  // exclusive popcount prefix per word pair: thread tid takes pairs [tid*ppt, ...)
  const int ppt = (npair + NT - 1) / NT;
  const uint2* bm2 = reinterpret_cast<const uint2*>(bm);
  int mine = 0;
  for (int q = 0; q < ppt; ++q) {
    const int pi = tid * ppt + q;
    if (pi < npair) {
      const uint2 x = bm2[pi];
      mine += __popc(x.x) + __popc(x.y);
    }
  }
  long long ctot = 0;
  int run = (int)block_excl_scan<NT, long long>((long long)mine, red, &ctot);
  for (int q = 0; q < ppt; ++q) {
    const int pi = tid * ppt + q;
    if (pi < npair) {
      const uint2 x = bm2[pi];
      pw[pi] = (unsigned short)run;
      run += __popc(x.x) + __popc(x.y);
    }
  }
  int c = (int)ctot;
  const bool ok = c == cnt && c <= a.wg_cap;
  if (!ok && tid == 0) atomicOr(a.err, ERR_COUNT);
  __syncthreads();
  V* bv = reinterpret_cast<V*>(smem + a.off_bvals);
  int* br = reinterpret_cast<int*>(smem + a.off_brows);
  auto rank_of = [&](int r) {  // r relative to rlo, its bit set
    const int w = r >> 5;
    const uint2 pr = bm2[w >> 1];
    const unsigned odd = 0u - (unsigned)(w & 1);
    const unsigned word = pr.x ^ ((pr.x ^ pr.y) & odd);
    return (int)pw[w >> 1] + (int)((unsigned)__popc(pr.x) & odd) + __popc(word & ((1u << (r & 31)) - 1u));
  };
  if (ok && one) {
    // first entries store at their rank, then the others add
    int rk[EW];
#pragma unroll
    for (int t = 0; t < EW; ++t) {
      const int r = rows[t] - rlo;
      rk[t] = (unsigned)r < (unsigned)span ? rank_of(r) : 0;
    }
#pragma unroll
    for (int t = 0; t < EW; ++t)
      if (first[t]) {
        bv[rk[t]] = vals[t];
        br[rk[t]] = rows[t];
      }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < EW; ++t) {
      const int e = tid + NT * t;
      const int r = rows[t] - rlo;
      if (e < u && !first[t] && (unsigned)r < (unsigned)span) lds_add_cas<V>(&bv[rk[t]], vals[t]);
    }
  } else if (ok) {
    // more entries than registers: every entry adds into a zeroed staging area
    for (int s = tid; s < c; s += NT) bv[s] = V(0);
    __syncthreads();
    for (int cb = 0; cb < u; cb += NT * EW) {
#pragma unroll
      for (int t = 0; t < EW; ++t) {
        const int e = cb + tid + NT * t;
        if (e < u) {
          const int sg = seg_of(P, a.k, a.ktop, e);
          const int row = gload<int>(adj[sg] + 4LL * e);
          const V v = gload<V>(adjv[sg] + (long long)sizeof(V) * e);
          const int r = row - rlo;
          if ((unsigned)r < (unsigned)span) {
            const int rk = rank_of(r);
            br[rk] = row;  // every entry of a row writes the same row
            lds_add_cas<V>(&bv[rk], v);
          }
        }
      }
    }
  }
  __syncthreads();
  if (!ok) return;
  int* outr = a.out_r + o0;
  V* outv = (V*)a.out_v + o0;
  for (int e = tid; e < c; e += NT) {
    outr[e] = br[e];
    outv[e] = bv[e];
  }
}

// ---- host side ----

// 2^18 rows: 32 KiB of bitmap and 8 KiB of prefix, two workgroups per CU with the
// staging area (measured on R-MAT windows: 2^17 leaves more windows to the hash
// kernel, 2^19 halves the resident workgroups; both slower).
int bitmap_wg_span_max() { return 1 << 18; }

void lds_layout_bitmap_wg(bool numeric, int vbytes, int k, int span_max, int cap, KArgs& a) {
  auto align16 = [](int x) { return (x + 15) & ~15; };
  const int npair = (span_max + 63) >> 6;
  int off = npair * 8;  // bitmap words, two per pair
  a.off_bm = 0;
  a.off_pre = off;
  off = align16(off + npair * 2);
  if (numeric) {
    a.off_bvals = off;
    off = align16(off + cap * vbytes);
    a.off_brows = off;
    off = align16(off + cap * 4);
  } else {
    a.off_bvals = a.off_brows = 0;
  }
  a.off_P = off;
  off = (off + (k + 1) * 4 + 7) & ~7;
  a.off_adj = off;
  off += k * 8;
  a.off_adjv = off;
  if (numeric) off += k * 8;
  a.slice_bytes = align16(off);
  a.wg_span_max = span_max;
  a.wg_cap = cap;
}

template <bool NUM, typename V>
static hipError_t launch_bw(int bin, const KArgs& a, const int* list, int n, hipStream_t s) {
  const size_t lds = (size_t)a.slice_bytes;
  constexpr int EW = 8;  // 4096 (G2, windows) or 2048 (G1) entries in registers: at least cap_in
  if (bin == BIN_WIN)
    k_bitmap_wg<G2_THREADS, EW, NUM, true, V><<<n, G2_THREADS, lds, s>>>(a, list, n);
  else if (bin == BIN_G1)
    k_bitmap_wg<G1_THREADS, EW, NUM, false, V><<<n, G1_THREADS, lds, s>>>(a, list, n);
  else
    k_bitmap_wg<G2_THREADS, EW, NUM, false, V><<<n, G2_THREADS, lds, s>>>(a, list, n);
  return hipGetLastError();
}

hipError_t launch_bitmap_wg(int bin, bool numeric, bool f64, const KArgs& a, const int* d_list, int nunits,
                            hipStream_t s) {
  if (nunits <= 0) return hipSuccess;
  if (bin != BIN_G1 && bin != BIN_G2 && bin != BIN_WIN) return hipErrorInvalidValue;
  if (!numeric) return launch_bw<false, float>(bin, a, d_list, nunits, s);
  return f64 ? launch_bw<true, double>(bin, a, d_list, nunits, s) : launch_bw<true, float>(bin, a, d_list, nunits, s);
}

}  // namespace spk
