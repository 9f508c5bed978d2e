// Device body of the workgroup bitmap accumulator (bitmap_wg.hip: plain units;
// batch_fused.hip: the workgroup-sized columns of batched runs).
#pragma once
#include "wave_device.h"

namespace spk {

// One unit (a column, or a row window when WIN) of the unit's row range [rlo, rhi):
// the whole workgroup of NT threads.  `red` (NT / 64 + 1 entries) and `info` are
// workgroup-shared scratch; `smem` holds the layout of lds_layout_bitmap_wg.  A unit
// wider than a.wg_span_max rows is skipped (uniform: the caller's other kernel takes it).
// G: bitmap words per prefix entry (2, or 4 to halve the prefix's LDS where that
// lets more workgroups reside; a rank then counts up to three whole words).
template <int NT, int EW, bool NUM, bool WIN, typename V, int G = 2>
__device__ __forceinline__ void bitmap_wg_unit(const KArgs& a, unsigned char* smem, long long* red, int* info_p,
                                               int unit, int j, int blo, int rlo, int rhi) {
  int& info = *info_p;
  const int tid = threadIdx.x;
  const int span = rhi - rlo;
  if (span > a.wg_span_max) return;  // another kernel's unit (uniform)
  unsigned* bm = reinterpret_cast<unsigned*>(smem);
  static_assert(G == 2 || G == 4, "prefix groups of 2 or 4 words");
  static_assert(NT * EW <= SEG_MASK_UNITS, "the segment mask covers every in-register entry");
  unsigned short* pw = reinterpret_cast<unsigned short*>(smem + a.off_pre);  // set bits below each word group
  int* P = reinterpret_cast<int*>(smem + a.off_P);
  long long* adj = reinterpret_cast<long long*>(smem + a.off_adj);
  long long* adjv = reinterpret_cast<long long*>(smem + a.off_adjv);
  // the unit's output place (numeric), read now so that it arrives with the segment table
  int cnt = 0, o0 = 0;
  if (NUM) {
    if (WIN) {
      cnt = a.win_cnt[unit];
      o0 = a.colptr_c[j] + a.win_off[unit];
    } else {
      o0 = a.colptr_c[j];
      cnt = a.colptr_c[j + 1] - o0;
    }
  }
  unsigned char* sm = smem + a.off_mark;  // segment starts (a unit whose entries fit registers)
  if (tid < 64) {
    const int u = build_meta<NUM, V>(a, j, WIN, blo, P, adj, adjv);
    if (tid == 0) info = u;
    if (u <= NT * EW) build_seg_mask(P, a.k, u, sm);  // (uniform in this wavefront)
  }
  const int ngrp = (span + 32 * G - 1) / (32 * G);
  for (int w = tid; w < G * ngrp; w += NT) bm[w] = 0u;
  __syncthreads();
  const int u = info;
  const bool one = u <= NT * EW;  // every entry of the unit in registers at once
  auto seg_at = [&](int e) -> int { return one ? seg_fast(sm, e) : seg_of(P, a.k, a.ktop, e); };
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
        const int sg = seg_at(e);
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
  // exclusive popcount prefix per group of G words: thread tid takes groups
  // [tid*gpt, ...)
  const int gpt = (ngrp + NT - 1) / NT;
  const uint2* bm2 = reinterpret_cast<const uint2*>(bm);
  const uint4* bm4 = reinterpret_cast<const uint4*>(bm);
  auto group_pop = [&](int gi) {
    if (G == 2) {
      const uint2 x = bm2[gi];
      return __popc(x.x) + __popc(x.y);
    }
    const uint4 x = bm4[gi];
    return __popc(x.x) + __popc(x.y) + __popc(x.z) + __popc(x.w);
  };
  int mine = 0;
  for (int q = 0; q < gpt; ++q) {
    const int gi = tid * gpt + q;
    if (gi < ngrp) mine += group_pop(gi);
  }
  long long ctot = 0;
  int run = (int)block_excl_scan<NT, long long>((long long)mine, red, &ctot);
  for (int q = 0; q < gpt; ++q) {
    const int gi = tid * gpt + q;
    if (gi < ngrp) {
      pw[gi] = (unsigned short)run;
      run += group_pop(gi);
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
    const unsigned low = (1u << (r & 31)) - 1u;
    if (G == 2) {
      const uint2 pr = bm2[w >> 1];
      const unsigned odd = 0u - (unsigned)(w & 1);
      const unsigned word = pr.x ^ ((pr.x ^ pr.y) & odd);
      return (int)pw[w >> 1] + (int)((unsigned)__popc(pr.x) & odd) + __popc(word & low);
    }
    // whole words of the quad below word i, then the bits below r in word i (masks and
    // selects: no dynamic register indexing)
    const int i = w & 3;
    const uint4 x = bm4[w >> 2];
    const unsigned m0 = i > 0 ? ~0u : 0u, m1 = i > 1 ? ~0u : 0u, m2 = i > 2 ? ~0u : 0u;
    const unsigned word = i == 0 ? x.x : i == 1 ? x.y : i == 2 ? x.z : x.w;
    return (int)pw[w >> 2] + __popc(x.x & m0) + __popc(x.y & m1) + __popc(x.z & m2) + __popc(word & low);
  };
  if (ok && one) {
    // first entries store at their rank, then the others add
    int rk[EW];
#pragma unroll
    for (int t = 0; t < EW; ++t) {
      const int r = rows[t] - rlo;
      rk[t] = (unsigned)r < (unsigned)span ? rank_of(r) : 0;
    }
    if (a.wg_overlay) __syncthreads();  // (uniform) the staging area overlays the bitmap
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
    // more entries than registers: every entry adds into a zeroed staging area (with
    // the overlay layout it lies between this unit's bitmap and the prefix words)
    if (a.wg_overlay && ngrp * G * 4 > a.off_bvals) {  // (uniform; excluded by the window split)
      if (tid == 0) atomicOr(a.err, ERR_COUNT);
      return;
    }
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
    gstore_nt<int>((long long)(outr + e), br[e]);
    gstore_nt<V>((long long)(outv + e), bv[e]);
  }
}

}  // namespace spk
