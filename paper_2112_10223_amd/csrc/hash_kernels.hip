// Symbolic and numeric hash kernels (Algorithms 5-8), one unit of work per
// wavefront (short columns) or per workgroup (long columns and row windows).
//
// A unit is one output column j, or one row window [rlo, rhi) of column j (the
// sliding hash, Section III-B).  Its inputs are k row-sorted segments, one per
// input matrix, that are concatenated logically into u entries.  Entry e belongs to
// the segment s with P[s] <= e < P[s+1], where P is the exclusive prefix of the
// segment lengths.  The unit finds s by a binary search over P in LDS, and the
// address of the entry is then adj[s] + e * sizeof(elem).
//
// Symbolic (Algorithm 6): a key-only table in LDS, initialised to -1.  A row is
// claimed with compare-and-swap and linear probing; the unit counts first claims.
// Numeric (Algorithm 5): (key, value) tables in LDS.  The row is claimed or found,
// then the value is added with an LDS atomic add.  The valid slots are compacted,
// sorted by row with an LSD radix sort in LDS (stable ranks from per-digit lane
// masks), and written out coalesced.
#include <climits>

#include "hash_common.h"

namespace spk {

int alpha_to_q(float alpha) {
  int aq = (int)(alpha * 1024.0f + 0.5f);
  if (aq < 1) aq = 1;
  if (aq > 1024) aq = 1024;
  return aq;
}

int table_slots(int entries, int alpha_q) { return slots_for(entries, alpha_q); }

// ---------------------------------------------------------------------------
// Wave bins: one wavefront per column, E entries per lane (u <= 64 E).
// ---------------------------------------------------------------------------
template <int E>
__global__ __launch_bounds__(256) void k_sym_wave(KArgs a, const int* __restrict__ list, int nunits) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int unit = xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + w;
  if (unit >= nunits) return;  // no block-wide barriers in this kernel
  unsigned char* base = smem + w * a.slice_bytes;
  int* T = (int*)base;
  int* P = (int*)(base + a.off_P);
  long long* adj = (long long*)(base + a.off_adj);
  const int j = list[unit];
  const int u = build_meta<false, float>(a, j, false, 0, P, adj, nullptr);
  int TS = slots_for(u, a.alpha_q);
  if (TS > a.ts_max) TS = a.ts_max;
  for (int s = lane; s < TS; s += 64) T[s] = -1;
  wave_sync();
  int rows[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = lane + 64 * t;
    if (e < u) rows[t] = gload<int>(adj[seg_of(P, a.k, a.ktop, e)] + 4LL * e);
  }
  int newc = 0;
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = lane + 64 * t;
    if (e < u) newc += sym_insert(T, TS, rows[t], a.hash_mode, a.err);
  }
  const int cnt = wave_sum(newc);
  if (lane == 0) a.colcnt[j] = cnt;
}

template <int E, typename V>
__global__ __launch_bounds__(256) void k_num_wave(KArgs a, const int* __restrict__ list, int nunits) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int unit = xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + w;
  if (unit >= nunits) return;
  unsigned char* base = smem + w * a.slice_bytes;
  int* K = (int*)base;
  V* Vt = (V*)(base + a.ts_max * 4);
  int* hist = (int*)(base + a.off_hist);
  u64* match = (u64*)(base + a.off_match);
  int* P = (int*)(base + a.off_P);
  long long* adj = (long long*)(base + a.off_adj);
  long long* adjv = (long long*)(base + a.off_adjv);
  const int j = list[unit];
  const int u = build_meta<true, V>(a, j, false, 0, P, adj, adjv);
  const int o0 = a.colptr_c[j];
  const int cnt = a.colptr_c[j + 1] - o0;
  int TS = slots_for(cnt, a.alpha_q);
  if (TS > a.ts_max) TS = a.ts_max;
  for (int s = lane; s < TS; s += 64) {
    K[s] = -1;
    Vt[s] = V(0);
  }
  for (int d = lane; d < 256; d += 64) match[d] = 0ull;
  wave_sync();
  int rows[E];
  V vals[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = lane + 64 * t;
    if (e < u) {
      const int sg = seg_of(P, a.k, a.ktop, e);
      rows[t] = gload<int>(adj[sg] + 4LL * e);
      vals[t] = gload<V>(adjv[sg] + (long long)sizeof(V) * e);
    }
  }
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = lane + 64 * t;
    if (e < u) num_insert<V>(K, Vt, TS, rows[t], vals[t], a.hash_mode, a.err);
  }
  wave_sync();
  // compact the valid slots to K[0, c), in slot order, in place
  int c = 0;
  for (int s0 = 0; s0 < TS; s0 += 64) {
    const int s = s0 + lane;
    const int key = K[s];
    const V val = Vt[s];
    const bool valid = key != -1;
    const u64 bal = ballot(valid);
    wave_sync();
    if (valid) {
      const int pos = c + mbcnt(bal);
      K[pos] = key;
      Vt[pos] = val;
    }
    c += __popcll(bal);
    wave_sync();
  }
  if (c != cnt) {
    if (lane == 0) atomicOr(a.err, ERR_COUNT);
    if (c > cnt) c = cnt;
  }
  V* vs = Vt;
  const int in0 = a.unsorted ? 1 : wave_radix_sort<V>(K, Vt, K + TS / 2, Vt + TS / 2, c, 0, ceil_log2(a.m), hist, match, &vs);
  const int* ks = in0 ? K : K + TS / 2;
  int* outr = a.out_r + o0;
  V* outv = (V*)a.out_v + o0;
  for (int e = lane; e < c; e += 64) {
    gstore_nt<int>((long long)(outr + e), ks[e]);
    gstore_nt<V>((long long)(outv + e), vs[e]);
  }
}

// ---------------------------------------------------------------------------
// Workgroup bins and row windows: one workgroup of NT threads per unit.
// EW entries per thread are loaded before they are inserted; SPT bounds the
// table slots per thread (ts_max <= NT * SPT).
// ---------------------------------------------------------------------------
template <int NT, typename V>
__device__ __forceinline__ int block_radix_sort(int* K0, V* V0, int* K1, V* V1, int c, int rlo, int bits,
                                                int* histw, u64* matchw, long long* scratch, V** vres) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, tid = threadIdx.x;
  const int L = ((c + NW - 1) / NW + 63) & ~63;
  const int lo = min(c, w * L), hi = min(c, (w + 1) * L);
  int* h = histw + w * 256;
  u64* mt = matchw + w * 256;
  int* sk = K0;
  V* sv = V0;
  int* dk = K1;
  V* dv = V1;
  int in0 = 1;
  for (int sh = 0; sh < bits; sh += 8) {
    const int mask = bits - sh >= 8 ? 255 : (1 << (bits - sh)) - 1;
    reinterpret_cast<int4*>(h)[lane_id()] = make_int4(0, 0, 0, 0);
    wave_sync();
    for (int b0 = lo; b0 < hi; b0 += 64) {
      const int e = b0 + lane_id();
      if (e < hi) atomicAdd(&h[((sk[e] - rlo) >> sh) & mask], 1);
    }
    __syncthreads();
    int tot = 0;
    if (tid < 256) {
#pragma unroll
      for (int v = 0; v < NW; ++v) tot += histw[v * 256 + tid];
    }
    const long long ex = block_excl_scan<NT, long long>((long long)tot, scratch);
    if (tid < 256) {
      int run = (int)ex;
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        const int x = histw[v * 256 + tid];
        histw[v * 256 + tid] = run;
        run += x;
      }
    }
    __syncthreads();
    wave_scatter<V>(sk, sv, dk, dv, lo, hi, rlo, sh, mask, h, mt);
    __syncthreads();
    int* tk = sk; sk = dk; dk = tk;
    V* tv = sv; sv = dv; dv = tv;
    in0 ^= 1;
  }
  *vres = sv;
  return in0;
}

template <int NT, int EW, int SPT, bool NUM, bool WIN, typename V>
__global__ __launch_bounds__(NT) void k_hash_wg(KArgs a, const int* __restrict__ list, int nunits) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long red[NT / 64 + 1];
  __shared__ int info;
  const int unit = xcd_remap(blockIdx.x, gridDim.x);
  if (unit >= nunits) return;  // uniform over the block
  const int tid = threadIdx.x;
  int j, blo = 0, rlo = 0, rhi = a.m;
  if (WIN) {
    const int4 w = a.wrec[unit];
    j = w.x;
    rlo = w.y;
    rhi = w.z;
    blo = w.w;
  } else {
    j = list[unit];
  }
  if (rhi - rlo <= a.wg_span_max) return;  // the bitmap kernel's unit (uniform; wg_span_max = 0: none)
  int* K = (int*)smem;
  V* Vt = (V*)(smem + a.ts_max * 4);
  int* P = (int*)(smem + a.off_P);
  long long* adj = (long long*)(smem + a.off_adj);
  long long* adjv = (long long*)(smem + a.off_adjv);
  unsigned char* sm = smem + a.off_mark;
  if (tid < 64) {
    const int u = build_meta<NUM, V>(a, j, WIN, blo, P, adj, adjv);
    if (tid == 0) info = u;
    if (u <= SEG_MASK_UNITS) build_seg_mask(P, a.k, u, sm);  // (uniform in this wavefront)
  }
  int cnt = 0, o0 = 0, TS;
  if (NUM) {
    if (WIN) {
      cnt = a.win_cnt[unit];
      o0 = a.colptr_c[j] + a.win_off[unit];
    } else {
      o0 = a.colptr_c[j];
      cnt = a.colptr_c[j + 1] - o0;
    }
    TS = slots_for(cnt, a.alpha_q);
  }
  __syncthreads();
  const int u = info;
  if (!NUM) {
    const int bound = min(u, rhi - rlo);
    TS = slots_for(bound, a.alpha_q);
  }
  if (TS > a.ts_max) TS = a.ts_max;
  for (int s = tid; s < TS; s += NT) {
    K[s] = -1;
    if (NUM) Vt[s] = V(0);
  }
  if (NUM) {
    u64* matchw = (u64*)(smem + a.off_match);
    for (int d = tid; d < (NT / 64) * 256; d += NT) matchw[d] = 0ull;
  }
  __syncthreads();
  int newc = 0;
  for (int cb = 0; cb < u; cb += NT * EW) {
    int rows[EW];
    V vals[EW];
#pragma unroll
    for (int t = 0; t < EW; ++t) {
      const int e = cb + tid + NT * t;
      if (e < u) {
        const int sg = u <= SEG_MASK_UNITS ? seg_fast(sm, e) : seg_of(P, a.k, a.ktop, e);
        rows[t] = gload<int>(adj[sg] + 4LL * e);
        if (NUM) vals[t] = gload<V>(adjv[sg] + (long long)sizeof(V) * e);
      }
    }
#pragma unroll
    for (int t = 0; t < EW; ++t) {
      const int e = cb + tid + NT * t;
      if (e < u) {
        if (NUM) num_insert<V>(K, Vt, TS, rows[t], vals[t], a.hash_mode, a.err);
        else newc += sym_insert(K, TS, rows[t], a.hash_mode, a.err);
      }
    }
  }
  __syncthreads();
  if (!NUM) {
    const long long total = block_sum<NT, long long>((long long)newc, red);
    if (tid == 0) {
      if (WIN) a.win_cnt[unit] = (int)total;
      else a.colcnt[j] = (int)total;
    }
    return;
  }
  // compaction of the valid slots to K[0, c); the slots are staged in registers
  // so that no thread overwrites a slot another thread has not read yet
  int keys[SPT];
  V vv[SPT];
  int nv = 0;
#pragma unroll
  for (int t = 0; t < SPT; ++t) {
    const int s = t * NT + tid;
    keys[t] = s < TS ? K[s] : -1;
    vv[t] = s < TS ? Vt[s] : V(0);
    nv += keys[t] != -1;
  }
  long long ctot = 0;
  int pos = (int)block_excl_scan<NT, long long>((long long)nv, red, &ctot);
#pragma unroll
  for (int t = 0; t < SPT; ++t) {
    if (keys[t] != -1) {
      K[pos] = keys[t];
      Vt[pos] = vv[t];
      ++pos;
    }
  }
  __syncthreads();
  int c = (int)ctot;
  if (c != cnt) {
    if (tid == 0) atomicOr(a.err, ERR_COUNT);
    if (c > cnt) c = cnt;
  }
  V* vs = Vt;
  const int in0 = a.unsorted ? 1
                             : block_radix_sort<NT, V>(K, Vt, K + TS / 2, Vt + TS / 2, c, rlo, ceil_log2(rhi - rlo),
                                                       (int*)(smem + a.off_hist), (u64*)(smem + a.off_match), red,
                                                       &vs);
  const int* ks = in0 ? K : K + TS / 2;
  int* outr = a.out_r + o0;
  V* outv = (V*)a.out_v + o0;
  for (int e = tid; e < c; e += NT) {
    gstore_nt<int>((long long)(outr + e), ks[e]);
    gstore_nt<V>((long long)(outv + e), vs[e]);
  }
}

// ---------------------------------------------------------------------------
// Host side: LDS layouts and launches.
// ---------------------------------------------------------------------------
static inline int align_up(int x, int a) { return (x + a - 1) / a * a; }

static bool is_wave_bin(int b) { return b >= BIN_W1 && b <= BIN_W16; }

int bin_threads(int bin) {
  if (is_wave_bin(bin)) return 256;
  if (bin == BIN_G1) return G1_THREADS;
  return G2_THREADS;
}

int bin_units_per_block(int bin) { return is_wave_bin(bin) ? WAVES_PER_BLOCK : 1; }

void lds_layout(int bin, bool numeric, int vbytes, int k, int ts_max, KArgs& a) {
  const int nw = bin_threads(bin) / 64;
  int off = ts_max * 4;
  if (numeric) off += ts_max * vbytes;
  off = align_up(off, 16);
  if (numeric) {
    a.off_hist = off;
    off += (is_wave_bin(bin) ? 1 : nw) * 256 * 4;
    a.off_match = off;
    off += (is_wave_bin(bin) ? 1 : nw) * 256 * 8;
  } else {
    a.off_hist = a.off_match = 0;
  }
  a.off_P = off;
  off = align_up(off + (k + 1) * 4, 8);
  a.off_adj = off;
  off += k * 8;
  a.off_adjv = off;
  if (numeric) off += k * 8;
  if (!is_wave_bin(bin)) {  // workgroup units: the segment-start mask
    off = align_up(off, 16);
    a.off_mark = off;
    off += seg_mask_bytes(k);
  }
  a.slice_bytes = align_up(off, 16);
  a.ts_max = ts_max;
}

int max_lds_bytes() { return 160 * 1024; }

template <typename V>
static hipError_t launch_num(int bin, const KArgs& a, const int* list, int n, hipStream_t s) {
  const int blocks_wave = (n + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  const size_t lds_wave = (size_t)a.slice_bytes * WAVES_PER_BLOCK;
  const size_t lds = (size_t)a.slice_bytes;
  switch (bin) {
    case BIN_W1: k_num_wave<1, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W2: k_num_wave<2, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W3: k_num_wave<3, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W4: k_num_wave<4, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W5: k_num_wave<5, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W6: k_num_wave<6, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W8: k_num_wave<8, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W10: k_num_wave<10, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W12: k_num_wave<12, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W16: k_num_wave<16, V><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_G1: k_hash_wg<G1_THREADS, 4, 16, true, false, V><<<n, G1_THREADS, lds, s>>>(a, list, n); break;
    case BIN_G2: k_hash_wg<G2_THREADS, 4, 32, true, false, V><<<n, G2_THREADS, lds, s>>>(a, list, n); break;
    case BIN_WIN: k_hash_wg<G2_THREADS, 4, 32, true, true, V><<<n, G2_THREADS, lds, s>>>(a, list, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_sym(int bin, const KArgs& a, const int* list, int n, hipStream_t s) {
  const int blocks_wave = (n + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  const size_t lds_wave = (size_t)a.slice_bytes * WAVES_PER_BLOCK;
  const size_t lds = (size_t)a.slice_bytes;
  switch (bin) {
    case BIN_W1: k_sym_wave<1><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W2: k_sym_wave<2><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W3: k_sym_wave<3><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W4: k_sym_wave<4><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W5: k_sym_wave<5><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W6: k_sym_wave<6><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W8: k_sym_wave<8><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W10: k_sym_wave<10><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W12: k_sym_wave<12><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_W16: k_sym_wave<16><<<blocks_wave, 256, lds_wave, s>>>(a, list, n); break;
    case BIN_G1: k_hash_wg<G1_THREADS, 8, 1, false, false, float><<<n, G1_THREADS, lds, s>>>(a, list, n); break;
    case BIN_G2: k_hash_wg<G2_THREADS, 8, 1, false, false, float><<<n, G2_THREADS, lds, s>>>(a, list, n); break;
    case BIN_WIN: k_hash_wg<G2_THREADS, 8, 1, false, true, float><<<n, G2_THREADS, lds, s>>>(a, list, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_hash(int bin, bool numeric, bool f64, const KArgs& a, const int* d_list, int nunits,
                       hipStream_t s) {
  if (nunits <= 0) return hipSuccess;
  if (!numeric) return launch_sym(bin, a, d_list, nunits, s);
  return f64 ? launch_num<double>(bin, a, d_list, nunits, s) : launch_num<float>(bin, a, d_list, nunits, s);
}

const char* hash_kernel_name(int bin, bool numeric) {
  static const char* sym[NBINS] = {"empty", "sym_wave_e1", "sym_wave_e2", "sym_wave_e3", "sym_wave_e4",
                                   "sym_wave_e5", "sym_wave_e6", "sym_wave_e8", "sym_wave_e10", "sym_wave_e12",
                                   "sym_wave_e16", "sym_wg256", "sym_wg512", "sym_window"};
  static const char* num[NBINS] = {"empty", "num_wave_e1", "num_wave_e2", "num_wave_e3", "num_wave_e4",
                                   "num_wave_e5", "num_wave_e6", "num_wave_e8", "num_wave_e10", "num_wave_e12",
                                   "num_wave_e16", "num_wg256", "num_wg512", "num_window"};
  return (bin >= 0 && bin < NBINS) ? (numeric ? num[bin] : sym[bin]) : "?";
}

}  // namespace spk
