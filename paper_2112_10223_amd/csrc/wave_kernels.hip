// Wave-bin kernels with a per-wavefront pipeline over consecutive columns.
//
// One wavefront owns `upw` consecutive units (columns) of a bin.  While it
// accumulates column t in its LDS table, the column pointers of column t+2 and the
// row (and value) loads of column t+1 are already in flight.  The two register
// sets alternate, and the loop is unrolled by two so that no register copy forces
// a wait.  Lane i < k keeps the base pointers of input i for the whole run
// (k <= 64).
//
// Symbolic (Algorithm 6): compare-and-swap claims in a key-only LDS table.  All
// E entries of a lane are claimed together, then the colliding ones probe on.
// Numeric (Algorithm 5): the same claims on (key, value) tables plus LDS atomic
// adds.  The table is then read into registers and bucketed by the top 8 bits of
// (row - min row).  Each entry is ranked inside its bucket by counting the smaller
// keys; rows are unique, so the bucket order needs no stability.  The sorted column
// is written out coalesced.
#include "hash_common.h"

namespace spk {

// Entry addresses of one unit: lockstep binary searches over the segment prefix P
// (all E searches advance together, one LDS round trip per step).
template <int E, bool NUM, typename V>
__device__ __forceinline__ void issue_unit_loads(const KArgs& a, const int* P, const long long* adj,
                                                 const long long* adjv, int u, int (&rows)[E], V (&vals)[E]) {
  const int lane = lane_id();
  int seg[E];
#pragma unroll
  for (int t = 0; t < E; ++t) seg[t] = 0;
  for (int step = a.ktop; step > 0; step >>= 1) {
    int pv[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int c = seg[t] + step;
      pv[t] = P[c < a.k ? c : a.k - 1];
    }
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int c = seg[t] + step;
      const int e = min(lane + 64 * t, u - 1);
      if (c < a.k && pv[t] <= e) seg[t] = c;
    }
  }
  long long ar[E], av[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    ar[t] = adj[seg[t]];
    if (NUM) av[t] = adjv[seg[t]];
  }
  const long long dummy = (long long)a.dummy;
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = min(lane + 64 * t, u - 1);  // masked lanes re-read the unit's last entry
    rows[t] = gload<int>(u > 0 ? ar[t] + 4LL * e : dummy);
    if (NUM) vals[t] = gload<V>(u > 0 ? av[t] + (long long)sizeof(V) * e : dummy);
  }
}

// Column pointers of unit column j: lane i < k reads colptr_i[j], colptr_i[j+1];
// lanes 0 and 1 also read colptr(B)[j], colptr(B)[j+1] for the numeric pass.
// Lanes >= k hold the pointer of input k-1 and so repeat lane k-1's reads; a null
// unit (j < 0) reads column 0 and is given zero length by build_unit_meta.
template <bool NUM>
__device__ __forceinline__ void issue_meta_loads(const KArgs& a, long long cpp, int j, int& s, int& e, int& cc) {
  const int lane = lane_id();
  const int jj = j < 0 ? 0 : j;
  s = gload<int>(cpp + 4LL * jj);
  e = gload<int>(cpp + 4LL * (jj + 1));
  if (NUM) cc = gload<int>((long long)(a.colptr_c + jj + (lane & 1)));
}

// Segment table of a unit from its column pointers; returns u.
template <bool NUM, typename V>
__device__ __forceinline__ int build_unit_meta(const KArgs& a, long long rip, long long vap, int s, int e, int* P,
                                               long long* adj, long long* adjv, bool null_unit) {
  const int lane = lane_id();
  const int len = (lane < a.k && !null_unit) ? e - s : 0;
  const int incl = wave_scan_add(len);
  const int ex = incl - len;
  if (lane < a.k) {
    P[lane] = ex;
    adj[lane] = rip + 4LL * (s - ex);
    if (NUM) adjv[lane] = vap + (long long)sizeof(V) * (s - ex);
  }
  return readlane(incl, 63);
}

// Algorithm 6 on E entries per lane with batched claims; returns this lane's new keys.
template <int E>
__device__ __forceinline__ int sym_insert_batch(int* T, int TS, int mode, int u, const int (&rows)[E], int* err) {
  const int lane = lane_id();
  int slot[E];
  bool act[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    act[t] = lane + 64 * t < u;
    slot[t] = hash_slot(rows[t], TS, mode);
  }
  int newc = 0;
  for (int probe = 0; probe < TS; ++probe) {
    int old[E];
#pragma unroll
    for (int t = 0; t < E; ++t) old[t] = act[t] ? atomicCAS(&T[slot[t]], -1, rows[t]) : -2;
    bool more = false;
#pragma unroll
    for (int t = 0; t < E; ++t) {
      if (act[t]) {
        if (old[t] == -1) {
          ++newc;
          act[t] = false;
        } else if (old[t] == rows[t]) {
          act[t] = false;
        } else {
          slot[t] = slot[t] + 1 == TS ? 0 : slot[t] + 1;
          more = true;
        }
      }
    }
    if (ballot(more) == 0) return newc;
  }
  atomicOr(err, ERR_PROBE);
  return newc;
}

// Algorithm 5 on E entries per lane with batched claims.
template <int E, typename V>
__device__ __forceinline__ void num_insert_batch(int* K, V* Vt, int TS, int mode, int u, const int (&rows)[E],
                                                 const V (&vals)[E], int* err) {
  const int lane = lane_id();
  int slot[E];
  bool act[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    act[t] = lane + 64 * t < u;
    slot[t] = hash_slot(rows[t], TS, mode);
  }
  for (int probe = 0; probe < TS; ++probe) {
    int old[E];
#pragma unroll
    for (int t = 0; t < E; ++t) old[t] = act[t] ? atomicCAS(&K[slot[t]], -1, rows[t]) : -2;
    bool more = false;
#pragma unroll
    for (int t = 0; t < E; ++t) {
      if (act[t]) {
        if (old[t] == -1 || old[t] == rows[t]) {
          atomicAdd(&Vt[slot[t]], vals[t]);
          act[t] = false;
        } else {
          slot[t] = slot[t] + 1 == TS ? 0 : slot[t] + 1;
          more = true;
        }
      }
    }
    if (ballot(more) == 0) return;
  }
  atomicOr(err, ERR_PROBE);
}

// Numeric work of one unit: table, accumulation, bucket-rank sort, write-out.
template <int E, typename V>
__device__ __forceinline__ void num_unit(const KArgs& a, unsigned char* base, int u, int cnt, int o0,
                                         const int (&rows)[E], const V (&vals)[E]) {
  constexpr int NCH = 2 * E;  // table chunks of 64 slots at load factor 1/2
  const int lane = lane_id();
  int* K = (int*)base;
  V* Vt = (V*)(base + a.ts_max * 4);
  int* hist = (int*)(base + a.off_hist);
  int TS = slots_for(cnt, a.alpha_q);
  if (TS > NCH * 64) TS = NCH * 64;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int s = 64 * c + lane;
    if (s < TS) {
      K[s] = -1;
      Vt[s] = V(0);
    }
  }
  reinterpret_cast<int4*>(hist)[lane] = make_int4(0, 0, 0, 0);
  wave_sync();
  num_insert_batch<E, V>(K, Vt, TS, a.hash_mode, u, rows, vals, a.err);
  wave_sync();
  int kk[NCH];
  V vv[NCH];
  int mn = INT_MAX, mx = -1;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int s = 64 * c + lane;
    kk[c] = s < TS ? K[s] : -1;
    vv[c] = s < TS ? Vt[s] : V(0);
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (kk[c] >= 0) {
      mn = min(mn, kk[c]);
      mx = max(mx, kk[c]);
    }
  }
  mn = wave_total_min(mn);
  mx = wave_total_max(mx);
  const int bits = mx >= mn ? ceil_log2(mx - mn + 1) : 0;
  const int sh = bits > 8 ? bits - 8 : 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c)
    if (kk[c] >= 0) atomicAdd(&hist[(kk[c] - mn) >> sh], 1);
  wave_sync();
  {
    const int4 h = reinterpret_cast<int4*>(hist)[lane];
    const int tot = h.x + h.y + h.z + h.w;
    const int ex = wave_scan_add(tot) - tot;
    wave_sync();
    reinterpret_cast<int4*>(hist)[lane] = make_int4(ex, ex + h.x, ex + h.x + h.y, ex + h.x + h.y + h.z);
  }
  wave_sync();
  // bucket scatter into K[0, c) (the table has been read into registers)
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (kk[c] >= 0) {
      const int p = atomicAdd(&hist[(kk[c] - mn) >> sh], 1);
      K[p] = kk[c];
      Vt[p] = vv[c];
    }
  }
  wave_sync();
  const int total = hist[255];
  if (total != cnt) {
    if (lane == 0) atomicOr(a.err, ERR_COUNT);
    cnt = 0;  // write nothing for this unit
  }
  // rank inside the bucket, place into K[TS/2 + .]
  const int half = TS / 2;
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int p = 64 * c + lane;
    if (p < cnt) {
      const int key = K[p];
      const V val = Vt[p];
      const int d = (key - mn) >> sh;
      const int be = hist[d];
      const int bs = d ? hist[d - 1] : 0;
      int r = 0;
      for (int q = bs; q < be; ++q) r += K[q] < key;
      K[half + bs + r] = key;
      Vt[half + bs + r] = val;
    }
  }
  wave_sync();
  // unconditional stores (masked-off lanes write the dummy area) keep the number of
  // memory operations per unit fixed, so the loads of the next unit stay in flight
  // lanes past the end repeat the last entry's store (same address, same value);
  // an empty unit writes into the dummy sink
  const long long dst = (long long)(a.out_r + o0), dsv = (long long)((V*)a.out_v + o0);
  const long long dmy = (long long)a.dummy + 2048 + 8LL * lane;  // write sink, never read
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int p = min(64 * c + lane, cnt - 1);
    const int q = p < 0 ? 0 : p;
    gstore<int>(cnt > 0 ? dst + 4LL * q : dmy, K[half + q]);
    gstore<V>(cnt > 0 ? dsv + (long long)sizeof(V) * q : dmy, Vt[half + q]);
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
// Units t >= nu are null units (no entries, no output): every step runs the same
// instruction sequence, so the compiler keeps the next unit's loads in flight.
template <int E, bool NUM, typename V>
__device__ __forceinline__ void pipe_step(const KArgs& a, unsigned char* base, int t, int nu, int ucol,
                                          long long cpp, long long rip, long long vap, int& ms, int& me, int& mc,
                                          UnitRegs<E, NUM, V>& cur, UnitRegs<E, NUM, V>& nxt) {
  const int lane = lane_id();
  {
    const int b = (t + 1) & 1;
    int* P = (int*)(base + a.off_P) + 64 * b;
    long long* adj = (long long*)(base + a.off_adj) + 64 * b;
    long long* adjv = (long long*)(base + a.off_adjv) + 64 * b;
    nxt.j = t + 1 < nu ? readlane(ucol, (t + 1) & 63) : -1;
    nxt.u = build_unit_meta<NUM, V>(a, rip, vap, ms, me, P, adj, adjv, nxt.j < 0);
    if (NUM) {
      nxt.o0 = readlane(mc, 0);
      nxt.cnt = nxt.j < 0 ? 0 : readlane(mc, 1) - nxt.o0;
    }
    issue_meta_loads<NUM>(a, cpp, t + 2 < nu ? readlane(ucol, (t + 2) & 63) : -1, ms, me, mc);
    wave_sync();
    issue_unit_loads<E, NUM, V>(a, P, adj, adjv, nxt.u, nxt.rows, nxt.vals);
  }
  if (NUM) {
    num_unit<E, V>(a, base, cur.u, cur.cnt, cur.o0, cur.rows, cur.vals);
  } else {
    int* T = (int*)base;
    int TS = slots_for(cur.u, a.alpha_q);
    if (TS > a.ts_max) TS = a.ts_max;
    for (int s = lane; s < TS; s += 64) T[s] = -1;
    wave_sync();
    const int newc = sym_insert_batch<E>(T, TS, a.hash_mode, cur.u, cur.rows, a.err);
    const int cnt = wave_total_add(newc);
    const long long dst = cur.j >= 0 ? (long long)(a.colcnt + cur.j) : (long long)a.dummy + 2048 + 8LL * lane;
    if (lane == 0) gstore<int>(dst, cnt);
    wave_sync();
  }
}

template <int E, bool NUM, typename V>
__global__ __launch_bounds__(256) void k_wave_pipe(KArgs a, const int* __restrict__ list, int nunits) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int gw = xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + w;
  const int ub = gw * a.upw;
  const int nu = min(a.upw, nunits - ub);
  if (nu <= 0) return;  // no block-wide barriers in this kernel
  unsigned char* base = smem + w * a.slice_bytes;
  const int li = lane < a.k ? lane : a.k - 1;
  const long long cpp = (long long)a.cp[li];
  const long long rip = (long long)a.ri[li];
  const long long vap = NUM ? (long long)a.va[li] : 0;
  const int ucol = lane < nu ? list[ub + lane] : 0;

  UnitRegs<E, NUM, V> A, B;
  int ms = 0, me = 0, mc = 0;
  // prologue: metadata and entry loads of unit 0, pointers of unit 1
  issue_meta_loads<NUM>(a, cpp, readlane(ucol, 0), ms, me, mc);
  {
    int* P = (int*)(base + a.off_P);
    long long* adj = (long long*)(base + a.off_adj);
    long long* adjv = (long long*)(base + a.off_adjv);
    A.u = build_unit_meta<NUM, V>(a, rip, vap, ms, me, P, adj, adjv, false);
    A.j = readlane(ucol, 0);
    if (NUM) {
      A.o0 = readlane(mc, 0);
      A.cnt = readlane(mc, 1) - A.o0;
    }
    issue_meta_loads<NUM>(a, cpp, nu > 1 ? readlane(ucol, 1) : -1, ms, me, mc);
    wave_sync();
    issue_unit_loads<E, NUM, V>(a, P, adj, adjv, A.u, A.rows, A.vals);
  }
  const int steps = (nu + 1) & ~1;
  for (int t = 0; t < steps; t += 2) {
    pipe_step<E, NUM, V>(a, base, t, nu, ucol, cpp, rip, vap, ms, me, mc, A, B);
    pipe_step<E, NUM, V>(a, base, t + 1, nu, ucol, cpp, rip, vap, ms, me, mc, B, A);
  }
}

// ---- host side ----
bool wave_pipe_ok(int k, int alpha_num_q) { return k <= 64 && alpha_num_q == 512; }

void lds_layout_pipe(int bin, bool numeric, int vbytes, int ts_max, KArgs& a) {
  int off = ts_max * 4;
  if (numeric) off += ts_max * vbytes;
  off = (off + 15) & ~15;
  a.off_hist = off;
  if (numeric) off += 256 * 4;
  a.off_P = off;
  off += 2 * 64 * 4;
  a.off_adj = off;
  off += 2 * 64 * 8;
  a.off_adjv = off;
  if (numeric) off += 2 * 64 * 8;
  a.slice_bytes = (off + 15) & ~15;
  a.ts_max = ts_max;
  (void)bin;
}

template <bool NUM, typename V>
static hipError_t launch_pipe_t(int bin, const KArgs& a, const int* list, int n, hipStream_t s) {
  const int waves = (n + a.upw - 1) / a.upw;
  const int blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  const size_t lds = (size_t)a.slice_bytes * WAVES_PER_BLOCK;
  switch (bin) {
    case BIN_W1: k_wave_pipe<1, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W2: k_wave_pipe<2, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W3: k_wave_pipe<3, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W4: k_wave_pipe<4, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W5: k_wave_pipe<5, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W6: k_wave_pipe<6, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W8: k_wave_pipe<8, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W10: k_wave_pipe<10, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W12: k_wave_pipe<12, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    case BIN_W16: k_wave_pipe<16, NUM, V><<<blocks, 256, lds, s>>>(a, list, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wave_pipe(int bin, bool numeric, bool f64, const KArgs& a, const int* d_list, int nunits,
                            hipStream_t s) {
  if (nunits <= 0) return hipSuccess;
  if (!numeric) return launch_pipe_t<false, float>(bin, a, d_list, nunits, s);
  return f64 ? launch_pipe_t<true, double>(bin, a, d_list, nunits, s)
             : launch_pipe_t<true, float>(bin, a, d_list, nunits, s);
}

}  // namespace spk
