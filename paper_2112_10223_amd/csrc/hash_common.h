// Shared pieces of the hash kernels: table sizing, the row hash, LDS inserts of
// Algorithms 5 and 6, the per-unit segment table, and the LDS radix sort.
#pragma once
#include <climits>

#include "device.h"
#include "internal.h"

namespace spk {

typedef unsigned long long u64;

// Table slots for `entries` keys at load factor alpha_q / 1024: a multiple of 64,
// at least 64.  Host and device use this same integer formula.
__host__ __device__ __forceinline__ int slots_for(long long entries, int alpha_q) {
  long long t = (entries * 1024 + alpha_q - 1) / alpha_q;
  t = (t + 63) & ~63LL;
  return (int)(t < 64 ? 64 : t);
}


// Hash of a row into [0, TS): the high bits of a multiplicative (Fibonacci) hash
// scaled to the table size.  The paper's hash is (a * r) & (2^q - 1) with a prime
// a; any choice gives the same result, only probe lengths differ.
__device__ __forceinline__ int hash_slot(int r, int TS, int mode) {
  if (mode) return 0;
  const uint32_t h = (uint32_t)r * 0x9E3779B1u;
  return (int)(((uint64_t)h * (uint32_t)TS) >> 32);
}

// Algorithm 6 (HashSymbolic) on one row: 1 if r was not stored yet.
__device__ __forceinline__ int sym_insert(int* T, int TS, int r, int mode, int* err) {
  int s = hash_slot(r, TS, mode);
  for (int probe = 0; probe < TS; ++probe) {
    const int old = atomicCAS(&T[s], -1, r);
    if (old == -1) return 1;
    if (old == r) return 0;
    s = (s + 1 == TS) ? 0 : s + 1;
  }
  atomicOr(err, ERR_PROBE);
  return 0;
}

// Value accumulation without LDS floating-point atomics (which are slow on this
// hardware): a compare-and-swap loop on the value's bit pattern.
template <typename V>
__device__ __forceinline__ void lds_add_cas(V* p, V v) {
  if constexpr (sizeof(V) == 4) {
    unsigned* q = reinterpret_cast<unsigned*>(p);
    unsigned old = *q;
    for (;;) {
      const unsigned nv = __float_as_uint(__uint_as_float(old) + (float)v);
      const unsigned prev = atomicCAS(q, old, nv);
      if (prev == old) break;
      old = prev;
    }
  } else {
    unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
    unsigned long long old = *q;
    for (;;) {
      const unsigned long long nv =
          (unsigned long long)__double_as_longlong(__longlong_as_double((long long)old) + (double)v);
      const unsigned long long prev = atomicCAS(q, old, nv);
      if (prev == old) break;
      old = prev;
    }
  }
}

// Algorithm 5 (HashAdd) on one entry.
template <typename V>
__device__ __forceinline__ void num_insert(int* K, V* Vt, int TS, int r, V v, int mode, int* err) {
  int s = hash_slot(r, TS, mode);
  for (int probe = 0; probe < TS; ++probe) {
    const int old = atomicCAS(&K[s], -1, r);
    if (old == -1 || old == r) {
      lds_add_cas<V>(&Vt[s], v);
      return;
    }
    s = (s + 1 == TS) ? 0 : s + 1;
  }
  atomicOr(err, ERR_PROBE);
}

// Segment table of a unit, built by one wavefront: P[i] (exclusive prefix of the
// segment lengths) and the adjusted base addresses of rows and values.  Returns u.
template <bool NUM, typename V>
__device__ __forceinline__ int build_meta(const KArgs& a, int j, bool win, int blo, int* P, long long* adj,
                                          long long* adjv) {
  const int lane = lane_id();
  int carry = 0;
  for (int base = 0; base < a.k; base += 64) {
    const int i = base + lane;
    int s = 0, e = 0;
    const int* rp = nullptr;
    const V* vp = nullptr;
    if (i < a.k) {
      // the row / value pointers are fetched together with the segment bounds
      rp = a.ri[i];
      if (NUM) vp = (const V*)a.va[i];
      if (win) {
        s = a.bpos[(long long)blo * a.k + i];
        e = max(a.bpos[(long long)(blo + 1) * a.k + i], s);  // (only an unsorted input could invert them)
      } else {
        const int* c = a.cp[i];
        s = c[j];
        e = c[j + 1];
      }
    }
    const int len = e - s;
    const int incl = wave_incl_scan(len);
    const int ex = carry + incl - len;
    if (i < a.k) {
      P[i] = ex;
      adj[i] = (long long)(rp + s) - 4LL * ex;
      if (NUM) adjv[i] = (long long)(vp + s) - (long long)sizeof(V) * ex;
    }
    carry += wave_bcast(incl, 63);
  }
  return carry;
}

// Segment holding concatenated entry e: the largest s < k with P[s] <= e.
__device__ __forceinline__ int seg_of(const int* P, int k, int ktop, int e) {
  int lo = 0;
  for (int step = ktop; step > 0; step >>= 1) {
    const int c = lo + step;
    if (c < k && P[c] <= e) lo = c;
  }
  return lo;
}

// Segment lookup in O(1) for a unit of at most SEG_MASK_UNITS entries: the starts of
// its non-empty segments are bits of a 64-word mask over the entry positions; entry e
// lies in the non-empty segment numbered (starts at positions <= e) - 1, which nzmap
// turns into the input.  Layout at `m` (seg_mask_bytes(k)): mask, per-word prefix
// counts (64 ints), nzmap (k ints).  Built by one wavefront after build_meta wrote P.
constexpr int SEG_MASK_UNITS = 64 * 64;
__host__ __device__ constexpr int seg_mask_bytes(int k) { return 64 * 8 + 64 * 4 + k * 4; }

__device__ __forceinline__ void build_seg_mask(const int* P, int k, int u, unsigned char* m) {
  unsigned long long* smask = reinterpret_cast<unsigned long long*>(m);
  int* mpre = reinterpret_cast<int*>(m + 64 * 8);
  int* nzmap = mpre + 64;
  const int lane = lane_id();
  smask[lane] = 0ull;
  wave_sync();
  int rc = 0;
  for (int base = 0; base < k; base += 64) {
    const int i = base + lane;
    int s0 = 0, s1 = 0;
    if (i < k) {
      s0 = P[i];
      s1 = i + 1 < k ? P[i + 1] : u;
    }
    const int nz = s1 > s0 ? 1 : 0;
    const int incl = wave_scan_add(nz);
    if (nz) {
      atomicOr(&smask[s0 >> 6], 1ull << (s0 & 63));
      nzmap[rc + incl - 1] = i;
    }
    rc += readlane(incl, 63);
  }
  wave_sync();
  const int cw = __popcll(smask[lane]);
  mpre[lane] = wave_scan_add(cw) - cw;
}

__device__ __forceinline__ int seg_fast(const unsigned char* m, int e) {
  const unsigned long long* smask = reinterpret_cast<const unsigned long long*>(m);
  const int* mpre = reinterpret_cast<const int*>(m + 64 * 8);
  const int w = e >> 6, b = e & 63;
  const unsigned long long upto = b == 63 ? ~0ull : (2ull << b) - 1ull;
  return mpre[64 + mpre[w] + (int)__popcll(smask[w] & upto) - 1];
}

// One LSD pass over src[lo, hi) of a wavefront: stable scatter into dst by the digit
// ((key - rlo) >> sh) & mask.  `off` holds the running output offset per digit.
// `match` (256 lane masks) must be all zero on entry and is all zero on exit.
template <typename V>
__device__ __forceinline__ void wave_scatter(const int* sk, const V* sv, int* dk, V* dv, int lo, int hi, int rlo,
                                             int sh, int mask, int* off, u64* match) {
  const int lane = lane_id();
  const u64 lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int b0 = lo; b0 < hi; b0 += 64) {
    const int e = b0 + lane;
    const bool valid = e < hi;
    int key = 0, d = 0;
    V val = 0;
    if (valid) {
      key = sk[e];
      val = sv[e];
      d = ((key - rlo) >> sh) & mask;
      atomicOr(&match[d], 1ull << lane);
    }
    wave_sync();
    u64 mm = 0;
    int o = 0;
    if (valid) {
      mm = match[d];
      o = off[d];
    }
    wave_sync();
    if (valid) {
      const int rank = __popcll(mm & lt);
      dk[o + rank] = key;
      dv[o + rank] = val;
      if (rank == 0) {
        off[d] = o + __popcll(mm);
        match[d] = 0ull;
      }
    }
    wave_sync();
  }
}

// Radix sort of c unique keys (and values) by (key - rlo), `bits` significant bits,
// by one wavefront.  Ping-pongs between (K0,V0) and (K1,V1); returns the buffer
// holding the result.
template <typename V>
__device__ __forceinline__ int wave_radix_sort(int* K0, V* V0, int* K1, V* V1, int c, int rlo, int bits,
                                               int* hist, u64* match, V** vres) {
  const int lane = lane_id();
  int* sk = K0;
  V* sv = V0;
  int* dk = K1;
  V* dv = V1;
  int in0 = 1;
  for (int sh = 0; sh < bits; sh += 8) {
    const int mask = bits - sh >= 8 ? 255 : (1 << (bits - sh)) - 1;
    reinterpret_cast<int4*>(hist)[lane] = make_int4(0, 0, 0, 0);
    wave_sync();
    for (int b0 = 0; b0 < c; b0 += 64) {
      const int e = b0 + lane;
      if (e < c) atomicAdd(&hist[((sk[e] - rlo) >> sh) & mask], 1);
    }
    wave_sync();
    const int4 h = reinterpret_cast<int4*>(hist)[lane];
    const int tot = h.x + h.y + h.z + h.w;
    const int ex = wave_incl_scan(tot) - tot;
    wave_sync();
    reinterpret_cast<int4*>(hist)[lane] = make_int4(ex, ex + h.x, ex + h.x + h.y, ex + h.x + h.y + h.z);
    wave_sync();
    wave_scatter<V>(sk, sv, dk, dv, 0, c, rlo, sh, mask, hist, match);
    int* tk = sk; sk = dk; dk = tk;
    V* tv = sv; sv = dv; dv = tv;
    in0 ^= 1;
  }
  *vres = sv;
  return in0;
}

}  // namespace spk
