// Device code of the wave-bin kernels: one wavefront per column, with a
// per-wavefront pipeline over its columns.  Included by the plain launch
// (wave_kernels.hip) and the batched launch (batch_kernels.hip).
//
// Wavefront gw of a launch of G wavefronts takes the bin's units gw, gw + G,
// gw + 2G, ... (at most 64).  While it accumulates one column in LDS, the column
// pointers of the column after next and the row (and value) loads of the next
// column are already in flight.  Two register sets alternate, and the loop is
// unrolled by two so that no register copy forces a wait.  Lane i < k keeps the
// base pointers of input i for the whole run (k <= 64).
//
// Two accumulators, chosen per launch:
//  * hash (Algorithms 5 and 6): linear-probing LDS tables with compare-and-swap
//    claims; the numeric table is then compacted, bucketed by the top 8 bits of
//    (row - min row) and ranked inside each bucket, which sorts the column;
//  * bitmap: one bit per row of the matrix in LDS (the dense accumulator of
//    Algorithm 4 with the value array indexed by rank); the rank of a row among
//    the set bits is its output position, so the column comes out sorted with no
//    probing and no sort.
// Either way the sorted column is written out coalesced.
#pragma once
#include "hash_common.h"

namespace spk {

// Entry addresses of one unit.  The non-empty segments (inputs with entries in the
// column) are numbered in order, and each sets the bit of its start position in a
// 64 E-bit start mask.  The segment of position p is (#starts at positions <= p)
// - 1: per chunk of 64 positions, the starts of earlier chunks (a scalar count)
// plus mbcnt over the chunk's mask word.  Lanes past the end take the unit's last
// entry (every unit has u > 0), so no load is masked off.
template <int E, bool NUM, typename V>
__device__ __forceinline__ void issue_unit_loads(const KArgs& a, unsigned char* base, const long long* adj, int u,
                                                 int (&rows)[E], V (&vals)[E]) {
  const int lane = lane_id();
  const unsigned long long* sb = reinterpret_cast<const unsigned long long*>(base + a.off_mark);
  long long ar[E], av[E];
  int before = -1;  // starts in earlier chunks, minus one
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const unsigned long long w = sb[t];
    // (the builtin returns int: go through unsigned so the low word is not sign-extended)
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(w >> 32));
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)w);
    const unsigned long long S = ((unsigned long long)hi << 32) | (unsigned long long)lo;
    const int seg = before + (int)(S & 1ull) + mbcnt(S >> 1);
    before += __popcll(S);
    if constexpr (NUM) {  // (rows, values) pointer pairs: one 16-byte read
      const longlong2 pr = reinterpret_cast<const longlong2*>(adj)[seg];
      ar[t] = pr.x;
      av[t] = pr.y;
    } else {
      ar[t] = adj[seg];
    }
  }
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = min(lane + 64 * t, u - 1);
    rows[t] = gload<int>(ar[t] + 4LL * e);
    if (NUM) vals[t] = gload<V>(av[t] + (long long)sizeof(V) * e);
  }
}

// Column pointers of unit column j: lane i < k reads colptr_i[j], colptr_i[j+1];
// lanes 0 and 1 also read colptr(B)[j], colptr(B)[j+1] for the numeric pass.
// Lanes >= k hold the pointer of input k-1 and so repeat lane k-1's reads.
template <bool NUM>
__device__ __forceinline__ void issue_meta_loads(const KArgs& a, long long cpp, int j, int& s, int& e, int& cc) {
  const int lane = lane_id();
  s = gload<int>(cpp + 4LL * j);
  e = gload<int>(cpp + 4LL * (j + 1));
  if (NUM) cc = gload<int>((long long)(a.colptr_c + j + (lane & 1)));
}

// Segment table of a unit from its column pointers: the base pointers of the
// non-empty segments, shifted so that entry index (position in the unit) addresses
// them, in segment order, and the start mask.  Returns u.
template <int E, bool NUM, typename V>
__device__ __forceinline__ int build_unit_meta(const KArgs& a, unsigned char* base, long long rip, long long vap,
                                               int s, int e, long long* adj) {
  const int lane = lane_id();
  const int len = lane < a.k ? e - s : 0;
  const int incl = wave_scan_add(len);
  const int ex = incl - len;
  const int ord = mbcnt(ballot(len > 0));
  if (len > 0) {
    // numeric: (rows, values) pointer pairs in the 16-byte slots of adj (its region
    // holds 64 pairs there)
    if constexpr (NUM)
      reinterpret_cast<longlong2*>(adj)[ord] = make_longlong2(rip + 4LL * (s - ex), vap + (long long)sizeof(V) * (s - ex));
    else
      adj[ord] = rip + 4LL * (s - ex);
  }
  unsigned* sb = reinterpret_cast<unsigned*>(base + a.off_mark);
  if (lane < 2 * E) sb[lane] = 0u;
  wave_sync();
  if (len > 0) atomicOr(&sb[ex >> 5], 1u << (ex & 31));
  return readlane(incl, 63);
}


// Coalesced write-out of an output column staged in LDS (rows br[0..c), values
// bv[0..c), rows ascending) at offset o0 of rowidx(B) / values(B).  Lanes past the
// end repeat the last entry's store (same address, same value).  With c == 0 (a
// replayed or failed unit) every lane stores into the write sink instead.  The base
// pointers are the same for the whole wavefront, so only the offsets are per lane.
template <int E, typename V>
__device__ __forceinline__ void write_column(const KArgs& a, int o0, int c, const int* br, const V* bv) {
  const int lane = lane_id();
  const bool live = c > 0;
  int* ob = live ? a.out_r + o0 : reinterpret_cast<int*>((char*)a.dummy + 2048);
  V* ov = live ? (V*)a.out_v + o0 : reinterpret_cast<V*>((char*)a.dummy + 2048 + 64);
  const int last = live ? c - 1 : 0;
  // every staged entry is read before the first store (one LDS round trip)
  int rr[E];
  V vv[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int q = min(64 * t + lane, last);
    rr[t] = br[q];
    vv[t] = bv[q];
  }
  // uniform base (in scalar registers) + zero-extended 32-bit offset: no 64-bit
  // address arithmetic per lane
  const unsigned long long sob = uniform_u64((unsigned long long)ob);
  const unsigned long long sov = uniform_u64((unsigned long long)ov);
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const unsigned q = (unsigned)min(64 * t + lane, last);
    gstore_nt<int>((long long)(sob + (unsigned long long)(q * 4u)), rr[t]);
    gstore_nt<V>((long long)(sov + (unsigned long long)(q * (unsigned)sizeof(V))), vv[t]);
  }
}

// Algorithms 5 and 6 on E entries per lane of a wavefront-private table, with
// linear probing.  Every entry of the wavefront probes at once, one step per round:
// a lane's E compare-and-swaps are in flight together, and the wavefront waits for
// its longest probe sequence once rather than once per index t.  A row's probe
// sequence depends only on the row, so concurrent inserts of the same row meet in
// the same slot.  NUM: once every row has its slot, the lanes whose claims created
// slots store their values (plain stores), then the lanes that found their row
// already there add with a compare-and-swap loop.  SYM counts first claims.
// Returns this lane's new keys.
template <int E, bool NUM, typename V>
__device__ __forceinline__ int insert_batch(int* K, V* Vt, int TS, int mode, int u, const int (&rows)[E],
                                            const V (&vals)[E], int* err) {
  const int lane = lane_id();
  // per entry: slot in the low 16 bits (TS <= 2048), state above: 0 probing,
  // 1 claimed the slot, 2 found its row there, 3 no entry
  constexpr int SH = 16, MASK = (1 << SH) - 1;
  int code[E];
#pragma unroll
  for (int t = 0; t < E; ++t) code[t] = hash_slot(rows[t], TS, mode) | ((lane + 64 * t < u ? 0 : 3) << SH);
  for (int probe = 0; probe < TS; ++probe) {
    bool pending = false;
#pragma unroll
    for (int t = 0; t < E; ++t) {
      if ((code[t] >> SH) == 0) {
        const int sl = code[t] & MASK;
        const int old = atomicCAS(&K[sl], -1, rows[t]);
        if (old == -1) code[t] = sl | (1 << SH);
        else if (old == rows[t]) code[t] = sl | (2 << SH);
        else {
          code[t] = sl + 1 == TS ? 0 : sl + 1;
          pending = true;
        }
      }
    }
    if (ballot(pending) == 0) break;  // (uniform)
  }
  int newc = 0;
#pragma unroll
  for (int t = 0; t < E; ++t) {
    if ((code[t] >> SH) == 0) atomicOr(err, ERR_PROBE);  // a full table: sized wrong
    newc += (code[t] >> SH) == 1 ? 1 : 0;
  }
  if (NUM) {
#pragma unroll
    for (int t = 0; t < E; ++t)
      if ((code[t] >> SH) == 1) Vt[code[t] & MASK] = vals[t];
    wave_sync();
#pragma unroll
    for (int t = 0; t < E; ++t)
      if ((code[t] >> SH) == 2) lds_add_cas<V>(&Vt[code[t] & MASK], vals[t]);
    wave_sync();
  }
  return newc;
}

// Numeric work of one unit: table, accumulation, compaction, bucket-rank sort,
// write-out.  The key and value arrays have 64 extra sink slots after ts_max; lanes
// without an entry write there, so no store is predicated.
template <int E, typename V>
__device__ __forceinline__ void num_unit(const KArgs& a, unsigned char* base, int u, int cnt, int o0, bool live,
                                         const int (&rows)[E], const V (&vals)[E]) {
  constexpr int NCH = 2 * E;  // 64-slot table chunks at load factor 1/2
  constexpr int RANK_UNROLL = 4;
  const int lane = lane_id();
  int* K = (int*)base;
  V* Vt = (V*)(base + (a.ts_max + 64) * 4);
  int* hist = (int*)(base + a.off_hist);  // 256 buckets + sink
  const int sink = a.ts_max + lane;
  int TS = slots_for(cnt, a.alpha_q);
  if (TS > NCH * 64) TS = NCH * 64;
#pragma unroll
  for (int c = 0; c < NCH; ++c) K[64 * c + lane] = -1;
  reinterpret_cast<int4*>(hist)[lane] = make_int4(0, 0, 0, 0);
  wave_sync();
  insert_batch<E, true, V>(K, Vt, TS, a.hash_mode, u, rows, vals, a.err);
  wave_sync();
  // compaction of the valid slots to A = [0, nc), slot order
  int kk[NCH];
  V vv[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    kk[c] = K[64 * c + lane];
    vv[c] = Vt[64 * c + lane];
  }
  int nc = 0, mn = INT_MAX, mx = -1;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const bool ok = kk[c] != -1;
    const uint64_t m = ballot(ok);
    const int dst = ok ? nc + mbcnt(m) : sink;
    K[dst] = kk[c];
    Vt[dst] = vv[c];
    nc += __popcll(m);
    mn = min(mn, ok ? kk[c] : INT_MAX);
    mx = max(mx, ok ? kk[c] : -1);
  }
  if (nc != cnt) {
    if (lane == 0) atomicOr(a.err, ERR_COUNT);
    nc = 0;  // write nothing for this unit
  }
  if (!live) nc = 0;  // a replayed unit writes nothing
  if (a.unsorted) {  // (uniform) table order
    wave_sync();
    write_column<E, V>(a, o0, nc, K, Vt);
    return;
  }
  mn = wave_total_min(mn);
  mx = wave_total_max(mx);
  const int bits = mx >= mn ? ceil_log2(mx - mn + 1) : 0;
  const int sh = bits > 8 ? bits - 8 : 0;
  wave_sync();
  // bucket histogram of A (bucket = top 8 bits of key - mn)
  int ka[E], dg[E];
  V va[E];
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int p = 64 * c + lane;
    ka[c] = K[p];
    va[c] = Vt[p];
    dg[c] = p < nc ? (ka[c] - mn) >> sh : 256;
    atomicAdd(&hist[dg[c]], 1);
  }
  wave_sync();
  {
    const int4 h = reinterpret_cast<int4*>(hist)[lane];
    const int tot = h.x + h.y + h.z + h.w;
    const int ex = wave_scan_add(tot) - tot;
    wave_sync();
    reinterpret_cast<int4*>(hist)[lane] = make_int4(ex, ex + h.x, ex + h.x + h.y, ex + h.x + h.y + h.z);
  }
  wave_sync();
  // scatter into buckets, B = [half, half + nc)
  const int half = NCH * 32;
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int pos = atomicAdd(&hist[dg[c]], 1);
    const int dst = dg[c] < 256 ? half + pos : sink;
    K[dst] = ka[c];
    Vt[dst] = va[c];
  }
  wave_sync();
  // rank inside the bucket (rows are unique), final order into A
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int p = 64 * c + lane;
    const bool ok = p < nc;
    const int key = K[half + p];
    const V val = Vt[half + p];
    const int d = ok ? (key - mn) >> sh : 0;
    const int be = ok ? hist[d] : 0;
    const int bs = (ok && d) ? hist[d - 1] : 0;
    // the first RANK_UNROLL members of the bucket without a loop, the rest in one
    int r = 0;
#pragma unroll
    for (int q = 0; q < RANK_UNROLL; ++q) {
      const int x = K[half + min(bs + q, NCH * 64 - 1)];
      r += (bs + q < be && x < key) ? 1 : 0;
    }
    if (ballot(be - bs > RANK_UNROLL) != 0)
      for (int q = bs + RANK_UNROLL; q < be; ++q) r += K[half + q] < key;
    const int dst = ok ? bs + r : sink;
    K[dst] = key;
    Vt[dst] = val;
  }
  wave_sync();
  write_column<E, V>(a, o0, nc, K, Vt);
}

// ---------------------------------------------------------------------------
// Bitmap accumulator for dense columns: a row-indexed bitmap in LDS (the sparse
// accumulator of Algorithm 4, with the dense array replaced by one bit per row and
// the value array indexed by rank).  Symbolic: OR the rows in, count the bits.
// Numeric: OR the rows in (the atomic OR's old word tells which entry came first),
// prefix-popcount the bitmap, and use rank(row) = #set bits below it as the output
// position.  That gives sorted output with no hash probing and no sort.  A first
// entry stores its row and value at that position; a later entry of the same row
// adds with compare-and-swap.
// The bitmap holds bm_nq x 256 words (bm_nq x 8192 rows).
// ---------------------------------------------------------------------------
// Symbolic: OR the rows in; an OR that finds its bit clear counts a new row.  The
// bitmap is all zero on entry (cleared at the start of the run) and is left all
// zero: the words the unit touched are cleared again.
template <int E>
__device__ __forceinline__ int bm_sym_unit(const KArgs& a, unsigned char* base, int u, const int (&rows)[E]) {
  const int lane = lane_id();
  unsigned* bm = reinterpret_cast<unsigned*>(base + a.off_bm);
  int newc = 0;
  // lanes past the end hold a copy of the unit's last row and OR nothing
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const bool in = lane + 64 * t < u;
    const unsigned bit = in ? 1u << (rows[t] & 31) : 0u;
    const unsigned old = atomicOr(&bm[rows[t] >> 5], bit);
    newc += (in && (old & bit) == 0) ? 1 : 0;
  }
  wave_sync();
#pragma unroll
  for (int t = 0; t < E; ++t) bm[rows[t] >> 5] = 0u;
  wave_sync();
  return wave_total_add(newc);
}

template <int E, typename V>
__device__ __forceinline__ void bm_num_unit(const KArgs& a, unsigned char* base, int u, int cnt, int o0, bool live,
                                            const int (&rows)[E], const V (&vals)[E]) {
  const int lane = lane_id();
  uint4* bm4 = reinterpret_cast<uint4*>(base + a.off_bm);
  unsigned* bm = reinterpret_cast<unsigned*>(bm4);
  unsigned short* pw = reinterpret_cast<unsigned short*>(base + a.off_pre);  // set bits below each word pair
  V* bv = reinterpret_cast<V*>(base + a.off_bvals);  // may overlay the bitmap (used after the ranks)
  // rows follow the 64 (E + 1) staged values (a.off_brows; a constant distance, so
  // one address serves both)
  int* br = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(bv) + 64 * (E + 1) * sizeof(V));
  const int nq = a.bm_nq;
  for (int q = 0; q < nq; ++q) bm4[q * 64 + lane] = make_uint4(0u, 0u, 0u, 0u);
  wave_sync();
  bool first[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    // lanes past the end hold a copy of the unit's last row and OR nothing
    const bool in = lane + 64 * t < u;
    const unsigned bit = in ? 1u << (rows[t] & 31) : 0u;
    const unsigned old = atomicOr(&bm[rows[t] >> 5], bit);
    first[t] = in && (old & bit) == 0;
  }
  wave_sync();
  // exclusive popcount prefix per pair of words (ranks stay below 64 E <= 1024, so
  // 16 bits hold them); lane handles the 4 words (2 pairs) of group q*64 + lane.
  // Two bitmap rows share one scan, one in each 16-bit half: no partial sum exceeds
  // the column's distinct rows (<= 1024), so the halves never carry into each other.
  int carry = 0;
  for (int q = 0; q < nq; q += 2) {
    const bool two = q + 1 < nq;
    const uint4 x = bm4[q * 64 + lane];
    const uint4 y = two ? bm4[(q + 1) * 64 + lane] : make_uint4(0u, 0u, 0u, 0u);
    const int x01 = __popc(x.x) + __popc(x.y), nx = x01 + __popc(x.z) + __popc(x.w);
    const int y01 = __popc(y.x) + __popc(y.y), ny = y01 + __popc(y.z) + __popc(y.w);
    const int packed = nx | (ny << 16);
    const int incl = wave_scan_add(packed);
    const int ex = incl - packed;
    const int tot = readlane(incl, 63);
    const int px = carry + (ex & 0xffff);
    carry += tot & 0xffff;
    const int py = carry + (ex >> 16);
    carry += tot >> 16;
    unsigned* pw32 = reinterpret_cast<unsigned*>(pw);
    pw32[q * 64 + lane] = (unsigned)px | ((unsigned)(px + x01) << 16);
    if (two) pw32[(q + 1) * 64 + lane] = (unsigned)py | ((unsigned)(py + y01) << 16);
  }
  int c = carry;
  if (c != cnt) {
    if (lane == 0) atomicOr(a.err, ERR_COUNT);
    c = 0;
  }
  if (!live) c = 0;  // a replayed unit writes nothing
  wave_sync();
  // rank(row) = set bits below it = output position; the first entry of a row puts
  // the row and its value there, later entries of the row add their values
  // every lookup is issued before the first is used (one LDS round trip, not E)
  // (the word is picked by masking, not by a select: a select between two array
  // elements is turned into an indexed scratch access)
  int rk[E];
  unsigned plo[E], phi[E], pp[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int w = (lane + 64 * t < u ? rows[t] : 0) >> 5;
    const uint2 pr = reinterpret_cast<const uint2*>(bm)[w >> 1];
    plo[t] = pr.x;
    phi[t] = pr.y;
    pp[t] = pw[w >> 1];
  }
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int r = lane + 64 * t < u ? rows[t] : 0;
    const unsigned odd = 0u - (unsigned)((r >> 5) & 1);  // all ones for the second word of the pair
    const unsigned word = plo[t] ^ ((plo[t] ^ phi[t]) & odd);
    rk[t] = (int)pp[t] + (int)((unsigned)__popc(plo[t]) & odd) + __popc(word & ((1u << (r & 31)) - 1u));
  }
  wave_sync();  // the bitmap is read for the last time above
  // entries that are not first write into per-lane sink slots 64 E + lane
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int d = first[t] ? rk[t] : 64 * E + lane;
    bv[d] = vals[t];
    br[d] = rows[t];
  }
  wave_sync();
#pragma unroll
  for (int t = 0; t < E; ++t)
    if (lane + 64 * t < u && !first[t]) lds_add_cas<V>(&bv[rk[t]], vals[t]);
  wave_sync();
  write_column<E, V>(a, o0, c, br, bv);
}

// Marks the entry registers of a unit as needed here.  Called before the next
// unit's loads are issued: the compiler then waits for these loads with the
// previous unit's stores still in flight (stores count in vmcnt on this target,
// and a wait placed after newer loads would also wait for them).
template <int E, bool NUM, typename V>
__device__ __forceinline__ void require_loaded(const int (&rows)[E], const V (&vals)[E]) {
#pragma unroll
  for (int t = 0; t < E; ++t) {
    asm volatile("" ::"v"(rows[t]));
    if constexpr (NUM) asm volatile("" ::"v"(vals[t]));
  }
}

// Stores into the write sink as many store instructions as one pipeline step
// issues, so that the pipeline loop is entered with the same memory-counter history
// as its back edge (loads, then one unit's stores).  Otherwise the compiler merges
// the two histories at the loop head into a wait for every outstanding store.
template <int E, bool NUM, typename V>
__device__ __forceinline__ void prime_stores(const KArgs& a) {
  const int lane = lane_id();
  const long long dmy = (long long)a.dummy + 2048 + 8LL * lane;
  // (the empty asm statements keep the compiler from merging the repeated stores)
  if constexpr (NUM) {
#pragma unroll
    for (int t = 0; t < E; ++t) {
      gstore<int>(dmy, 0);
      asm volatile("" ::: "memory");
      gstore<V>(dmy, V(0));
      asm volatile("" ::: "memory");
    }
  } else {
    gstore<int>(dmy, 0);
  }
}

template <int E, bool NUM, typename V>
struct UnitRegs {
  int rows[E];
  V vals[E];
  int u, j, cnt, o0;
};

// One pipeline step: finish the metadata of unit t+1, start loads for units t+2
// (pointers) and t+1 (entries), then process unit t.
// Steps t >= nu (the loop runs an even count) replay the wavefront's last unit with
// its output sent to the write sink: every step runs the same instruction sequence
// on a real column, so the compiler keeps the next unit's loads in flight.
template <int E, bool NUM, typename V, bool BM>
__device__ __forceinline__ void pipe_step(const KArgs& a, unsigned char* base, int t, int nu, int ucol,
                                          long long cpp, long long rip, long long vap, int& ms, int& me, int& mc,
                                          UnitRegs<E, NUM, V>& cur, UnitRegs<E, NUM, V>& nxt) {
  const int lane = lane_id();
  require_loaded<E, NUM, V>(cur.rows, cur.vals);
  {
    // one segment table: a unit's pointers are read into registers in the step
    // that writes them
    long long* adj = (long long*)(base + a.off_adj);
    nxt.j = t + 1 < nu ? readlane(ucol, t + 1) : -1;  // -1: a replay, no output
    nxt.u = build_unit_meta<E, NUM, V>(a, base, rip, vap, ms, me, adj);
    if (NUM) {
      nxt.o0 = readlane(mc, 0);
      nxt.cnt = readlane(mc, 1) - nxt.o0;
    }
    issue_meta_loads<NUM>(a, cpp, readlane(ucol, min(t + 2, nu - 1)), ms, me, mc);
    wave_sync();
    issue_unit_loads<E, NUM, V>(a, base, adj, nxt.u, nxt.rows, nxt.vals);
  }
  if constexpr (NUM && BM) {
    bm_num_unit<E, V>(a, base, cur.u, cur.cnt, cur.o0, cur.j >= 0, cur.rows, cur.vals);
  } else if constexpr (NUM) {
    num_unit<E, V>(a, base, cur.u, cur.cnt, cur.o0, cur.j >= 0, cur.rows, cur.vals);
  } else if constexpr (BM) {
    const int cnt = bm_sym_unit<E>(a, base, cur.u, cur.rows);
    // one unconditional store instruction: lane 0 writes the count, the other
    // lanes (and replayed units) write into their write-sink slots
    const long long dmy = (long long)a.dummy + 2048 + 8LL * lane;
    gstore<int>(lane == 0 && cur.j >= 0 ? (long long)(a.colcnt + cur.j) : dmy, cnt);
    wave_sync();
  } else {
    int* T = (int*)base;
    int TS = slots_for(cur.u, a.alpha_q);
    if (TS > a.ts_max) TS = a.ts_max;
    for (int s = lane; s < TS; s += 64) T[s] = -1;
    wave_sync();
    const int newc = insert_batch<E, false, V>(T, nullptr, TS, a.hash_mode, cur.u, cur.rows, cur.vals, a.err);
    const int cnt = wave_total_add(newc);
    const long long dmy = (long long)a.dummy + 2048 + 8LL * lane;
    gstore<int>(lane == 0 && cur.j >= 0 ? (long long)(a.colcnt + cur.j) : dmy, cnt);
    wave_sync();
  }
}

// The pipeline over one wavefront's units: nu <= 64 unit column ids, lane t of
// ucol holding unit t.  Every unit has entries (u > 0).
template <int E, bool NUM, typename V, bool BM>
__device__ __forceinline__ void run_pipe(const KArgs& a, unsigned char* base, int nu, int ucol) {
  const int lane = lane_id();
  const int li = lane < a.k ? lane : a.k - 1;
  const long long cpp = (long long)a.cp[li];
  const long long rip = (long long)a.ri[li];
  const long long vap = NUM ? (long long)a.va[li] : 0;

  UnitRegs<E, NUM, V> A, B;
  int ms = 0, me = 0, mc = 0;
  // prologue: metadata and entry loads of unit 0, pointers of unit 1
  issue_meta_loads<NUM>(a, cpp, readlane(ucol, 0), ms, me, mc);
  {
    long long* adj = (long long*)(base + a.off_adj);
    A.u = build_unit_meta<E, NUM, V>(a, base, rip, vap, ms, me, adj);
    A.j = readlane(ucol, 0);
    if (NUM) {
      A.o0 = readlane(mc, 0);
      A.cnt = readlane(mc, 1) - A.o0;
    }
    issue_meta_loads<NUM>(a, cpp, readlane(ucol, min(1, nu - 1)), ms, me, mc);
    wave_sync();
    issue_unit_loads<E, NUM, V>(a, base, adj, A.u, A.rows, A.vals);
  }
  if constexpr (!NUM && BM) {  // the symbolic bitmap starts all zero and stays so
    uint4* bm4 = reinterpret_cast<uint4*>(base + a.off_bm);
    for (int q = 0; q < a.bm_nq; ++q) bm4[q * 64 + lane] = make_uint4(0u, 0u, 0u, 0u);
    wave_sync();
  }
  prime_stores<E, NUM, V>(a);
  const int steps = (nu + 1) & ~1;
  for (int t = 0; t < steps; t += 2) {
    pipe_step<E, NUM, V, BM>(a, base, t, nu, ucol, cpp, rip, vap, ms, me, mc, A, B);
    pipe_step<E, NUM, V, BM>(a, base, t + 1, nu, ucol, cpp, rip, vap, ms, me, mc, B, A);
  }
}

// LDS layout of one wavefront's slice (bytes).  Region 1: the hash table (keys + 64
// sink slots, then values and the 256-bucket histogram) or the bitmap (nq x 1 KiB)
// with its pair prefix (nq x 256 B); for the numeric bitmap the rows and values
// staged by rank overlay the bitmap when they fit in it.  Then the start mask
// (E 64-bit words) and the segment pointer table.
__host__ __device__ inline void pipe_layout(int E, bool numeric, int vbytes, int ts_max, int bm_nq, KArgs& a) {
  int hash_bytes = (ts_max + 64) * 4;
  if (numeric) hash_bytes += (ts_max + 64) * vbytes + 272 * 4;
  int bm_bytes = 0;
  a.bm_nq = bm_nq;
  if (bm_nq > 0) {
    a.off_bm = 0;
    a.off_pre = bm_nq * 256 * 4;
    const int staged = 64 * (E + 1) * (vbytes + 4);  // 64 E positions + 64 sink slots
    a.off_bvals = staged <= a.off_pre ? 0 : a.off_pre + bm_nq * 256;
    a.off_brows = a.off_bvals + 64 * (E + 1) * vbytes;
    bm_bytes = !numeric ? a.off_pre : staged <= a.off_pre ? a.off_pre + bm_nq * 256 : a.off_brows + 64 * (E + 1) * 4;
  }
  int off = bm_nq > 0 ? bm_bytes : hash_bytes;
  off = (off + 15) & ~15;
  a.off_hist = ((ts_max + 64) * 4 + (ts_max + 64) * vbytes + 15) & ~15;  // used by the hash layout only
  const int meta_bytes = ((8 * E + 15) & ~15) + (numeric ? 64 * 16 : 64 * 8);
  if (numeric && bm_nq > 0 && meta_bytes <= bm_nq * 256) {
    // The start mask and the segment table of the next unit are read (its loads
    // issued) before this unit writes its prefix words, and written again only after
    // the unit's ranks are read: they share the prefix region.
    a.off_mark = a.off_pre;
    a.off_P = a.off_adj = a.off_pre + ((8 * E + 15) & ~15);
    a.off_adjv = a.off_adj;
    a.slice_bytes = off;
    a.ts_max = ts_max;
    return;
  }
  a.off_mark = off;
  off += 8 * E;
  off = (off + 15) & ~15;
  a.off_P = off;
  a.off_adj = off;  // numeric: 64 (rows, values) pointer pairs; symbolic: 64 row pointers
  off += numeric ? 64 * 16 : 64 * 8;
  a.off_adjv = a.off_adj;  // (inside the pairs)
  a.slice_bytes = (off + 15) & ~15;
  a.ts_max = ts_max;
}

}  // namespace spk
