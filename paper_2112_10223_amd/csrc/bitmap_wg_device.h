// Device body of the workgroup bitmap accumulator (bitmap_wg.hip: plain units;
// batch_fused.hip: the workgroup-sized columns of batched runs).
#pragma once
#include "wave_device.h"

namespace spk {

// One unit (a column, or a row window when WIN) of the unit's row range [rlo, rhi):
// the whole workgroup of NT threads.  `red` (NT / 64 + 1 entries) and `info` are
// workgroup-shared scratch; `smem` holds the layout of lds_layout_bitmap_wg.  A unit
// wider than a.wg_span_max rows is skipped (uniform: the caller's other kernel takes it).
template <int NT, int EW, bool NUM, bool WIN, typename V>
__device__ __forceinline__ void bitmap_wg_unit(const KArgs& a, unsigned char* smem, long long* red, int* info_p,
                                               int unit, int j, int blo, int rlo, int rhi) {
  int& info = *info_p;
  const int tid = threadIdx.x;
  const int span = rhi - rlo;
  if (span > a.wg_span_max) return;  // another kernel's unit (uniform)
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

}  // namespace spk
