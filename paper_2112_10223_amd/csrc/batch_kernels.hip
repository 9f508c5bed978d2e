// Kernels of the batched launch (include/spkadd_batch.h): the columns of every
// request form one global worklist.  Global column g belongs to request r with
// col_base(r) <= g < col_base(r) + n_r.
//
//   k_batch_init    clears the per-request outcome and the counters (a kernel, so
//                   the run can be captured in a graph)
//   k_batch_bounds  u_j of every column (Section III-A) and its slot: empty, too
//                   large for a wavefront (u_j > wave_max), or (wave bin E, accumulator)
//   k_batch_slot_scan / k_batch_scatter  counting sort of the columns by slot;
//                   inside a slot the columns keep their global order, so each
//                   request's columns are contiguous
//   k_batch_wave    persistent wave kernels, one launch per (E, accumulator) (by
//                   default runs use k_batch_fused instead, one launch per pass): chunks
//                   of the slot's list, split into runs of one request, each run
//                   through the same per-wavefront pipeline as the plain launch
//   k_batch_scan    one workgroup per request: colptr(B_r), nnz(B_r), capacity check
#include <climits>

#include "batch_device.h"
#include "scan_device.h"

namespace spk {

// Wavefront bins of the batch (same E menu as the plain launch).
__device__ __forceinline__ int batch_wave_index(int u) {
  const int e = (u + 63) >> 6;
  return e <= 1 ? 0 : e <= 2 ? 1 : e <= 3 ? 2 : e <= 4 ? 3 : e <= 5 ? 4 : e <= 6 ? 5 : e <= 8 ? 6 : e <= 10 ? 7
       : e <= 12 ? 8 : 9;
}

// The request that global column g belongs to: the last r with col_base(r) <= g.
// `cbase` holds the requests' col_base in LDS when there are at most BATCH_LDS_REQS
// requests (a search through global memory waits for one load per step).
constexpr int BATCH_LDS_REQS = 1024;
__device__ __forceinline__ int request_of(const BatchReq* __restrict__ reqs, const int* cbase, int nreq, int g) {
  int lo = 0, hi = nreq - 1;
  if (nreq <= BATCH_LDS_REQS) {
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cbase[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
  } else {
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (reqs[mid].col_base <= g) lo = mid;
      else hi = mid - 1;
    }
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_batch_init(BatchArgs b) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  for (int r = t; r < b.max_reqs; r += gridDim.x * 256) {
    b.status[r] = 0;
    b.nnz[r] = 0;
  }
  if (t < 1024) reinterpret_cast<unsigned*>(const_cast<void*>(b.dummy))[t] = 0u;
  if (t == 0) *b.err = 0;
}

// Block c handles columns [c * b.chunk, (c + 1) * b.chunk) in steps of blockDim.x
// columns (up to 1024: a column's inputs are read in dependent rounds, so the columns
// of a block are taken side by side rather than one step after another).
__global__ __launch_bounds__(1024) void k_batch_bounds(BatchArgs b) {
  __shared__ int cnt[BSLOTS];
  __shared__ int wh[16][BSLOTS];
  __shared__ int cbase[BATCH_LDS_REQS];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int nt = (int)blockDim.x, nw = nt >> 6;
  const int nreq = b.hdr->nreq, total = b.hdr->total_cols;
  if (threadIdx.x < BSLOTS) cnt[threadIdx.x] = 0;
  if (nreq <= BATCH_LDS_REQS)
    for (int i = threadIdx.x; i < nreq; i += nt) cbase[i] = b.reqs[i].col_base;
  __syncthreads();
  const int c0 = blockIdx.x * b.chunk;
  for (int step = 0; step < b.chunk; step += nt) {
    const int g = c0 + step + threadIdx.x;
    int slot = -1, r = -1;
    if (g < total && step + (int)threadIdx.x < b.chunk) {
      r = request_of(b.reqs, cbase, nreq, g);
      const BatchReq& q = b.reqs[r];
      const int j = g - q.col_base;
      // 16 inputs per round; the next round's colptr pointers are loaded together with
      // this round's colptr entries (one memory round trip per round).  Global (not
      // generic) loads, so each wait covers only the memory counter.
      constexpr int G = 16;
      const long long cpt = (long long)q.cp;
      const int kq = q.k;
      long long u = 0;
      long long ptr[G];
#pragma unroll
      for (int t = 0; t < G; ++t) ptr[t] = gload<long long>(cpt + 8LL * min(t, kq - 1));
      for (int i0 = 0; i0 < kq; i0 += G) {
        int s[G], e[G];
#pragma unroll
        for (int t = 0; t < G; ++t) {
          s[t] = gload<int>(ptr[t] + 4LL * j);
          e[t] = gload<int>(ptr[t] + 4LL * (j + 1));
        }
        if (i0 + G < kq) {
#pragma unroll
          for (int t = 0; t < G; ++t) ptr[t] = gload<long long>(cpt + 8LL * min(i0 + G + t, kq - 1));
        }
#pragma unroll
        for (int t = 0; t < G; ++t)
          if (i0 + t < kq) u += (long long)(e[t] - s[t]);
      }
      b.req_of[g] = r;
      b.colcnt[g] = 0;
      if (u <= 0) {
        slot = BSLOT_EMPTY;
      } else if (u > b.wave_max && u <= b.wg_max && q.m <= BATCH_WG_SPAN) {
        slot = BSLOT_WG;
      } else if (u > b.wave_max) {
        slot = BSLOT_LARGE;  // (the request's outcome is set below, once per wavefront and request)
      } else {
        const int wi = batch_wave_index((int)u);
        const int E = wave_bin_E(BIN_W1 + wi);
        const bool bm = b.accum_mode != 1 && q.nq > 0 &&
                        (b.accum_mode == 2 || (float)q.nq <= b.bitmap_ratio * (float)E);
        slot = BSLOT_WAVE + 2 * wi + (bm ? 1 : 0);
      }
      b.slot[g] = (unsigned char)slot;
    }
    {
      // a request with many long columns would otherwise send one atomic per column
      // to the same word: the first lane of each run of one request's long columns
      // in the wavefront sets it
      const bool large = slot == BSLOT_LARGE;
      const uint64_t lm = ballot(large);
      const int rprev = __shfl_up(r, 1, 64);
      const bool prev_large = lane > 0 && ((lm >> (lane - 1)) & 1ull);
      if (large && !(prev_large && rprev == r)) atomicOr(&b.status[r], REQ_TOO_LARGE);
    }
    for (int s = 0; s < BSLOTS; ++s) {
      const uint64_t mk = ballot(slot == s);
      if (lane == 0) wh[w][s] = __popcll(mk);
    }
    __syncthreads();
    if (threadIdx.x < BSLOTS) {
      int add = 0;
      for (int v = 0; v < nw; ++v) add += wh[v][threadIdx.x];
      cnt[threadIdx.x] += add;
    }
    __syncthreads();
  }
  if (threadIdx.x < BSLOTS) b.hist[blockIdx.x * BSLOTS + threadIdx.x] = cnt[threadIdx.x];
}

// One block of 1024 threads; wavefront w scans slots w, w + 16, ... over the bounds
// blocks that hold columns of this run (the others find no columns).  Lane l of a
// wavefront takes a contiguous run of at most 16 blocks (there are at most
// BATCH_MAX_BOUNDS_BLOCKS = 1024), all its loads issued together.
__global__ __launch_bounds__(1024) void k_batch_slot_scan(BatchArgs b) {
  constexpr int MAXPER = BATCH_MAX_BOUNDS_BLOCKS / 64;
  __shared__ int tot[BSLOTS];
  const int lane = lane_id();
  const int total = b.hdr->total_cols;
  const int used = total > 0 ? (int)(((long long)total + b.chunk - 1) / b.chunk) : 0;
  const int nb = used < b.nblk ? used : b.nblk;
  const int per = (nb + 63) >> 6, b0 = lane * per;
  const int last = nb > 0 ? nb - 1 : 0;  // nblk >= 1: row 0 of hist always exists
  for (int s = threadIdx.x >> 6; s < BSLOTS; s += 16) {
    int v[MAXPER];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < MAXPER; ++i) {
      const int t = b0 + i;
      const bool mine = i < per && t < nb;
      const int x = b.hist[min(t, last) * BSLOTS + s];  // clamped index, no guard on the load
      v[i] = mine ? x : 0;
      sum += v[i];
    }
    const int incl = wave_scan_add(sum);
    int run = incl - sum;
#pragma unroll
    for (int i = 0; i < MAXPER; ++i) {
      const int t = b0 + i;
      if (i < per && t < nb) b.hist[t * BSLOTS + s] = run;
      run += v[i];
    }
    if (lane == 0) tot[s] = readlane(incl, 63);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int x = 0; x < BSLOTS; ++x) {
      b.slotoff[x] = acc;
      b.slotoff[BSLOTS + 1 + x] = tot[x];
      acc += tot[x];
    }
    b.slotoff[BSLOTS] = acc;
  }
}

__global__ __launch_bounds__(256) void k_batch_scatter(BatchArgs b) {
  __shared__ int run[BSLOTS];
  __shared__ int wc[4][BSLOTS];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int total = b.hdr->total_cols;
  if (threadIdx.x < BSLOTS) run[threadIdx.x] = b.slotoff[threadIdx.x] + b.hist[blockIdx.x * BSLOTS + threadIdx.x];
  __syncthreads();
  const int c0 = blockIdx.x * b.chunk;
  for (int step = 0; step < b.chunk; step += 256) {
    const int g = c0 + step + threadIdx.x;
    const int slot = g < total ? (int)b.slot[g] : -1;
    int rank = 0;
    for (int s = 0; s < BSLOTS; ++s) {
      const uint64_t mk = ballot(slot == s);
      if (slot == s) rank = mbcnt(mk);
      if (lane == 0) wc[w][s] = __popcll(mk);
    }
    __syncthreads();
    if (slot >= BSLOT_WAVE) {
      int before = 0;
      for (int v = 0; v < w; ++v) before += wc[v][slot];
      b.list[run[slot] + before + rank] = g;
    }
    __syncthreads();
    if (threadIdx.x < BSLOTS) run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] +
                                                   wc[3][threadIdx.x];
    __syncthreads();
  }
}

// Persistent, one launch per (wave bin, accumulator): wavefront gw of G takes chunks
// gw, gw + G, ... of its slot.
template <int E, bool NUM, typename V, bool BM>
__global__ __launch_bounds__(64 * PIPE_WAVES_PER_BLOCK) void k_batch_wave(BatchArgs b, KArgs a, int slot) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = threadIdx.x >> 6;
  const int G = (int)gridDim.x * PIPE_WAVES_PER_BLOCK;
  const int gw = xcd_remap(blockIdx.x, gridDim.x) * PIPE_WAVES_PER_BLOCK + w;
  slot_chunks<E, NUM, V, BM, false>(b, a, slot, smem + w * a.slice_bytes, gw, G);
}

// One workgroup per request: colptr(B_r) by an exclusive scan of its column counts.
__global__ __launch_bounds__(BATCH_SCAN_THREADS) void k_batch_scan(BatchArgs b) {
  __shared__ long long scratch[BATCH_SCAN_THREADS / 64 + 1];
  __shared__ int buf[BATCH_SCAN_THREADS * 16];
  const int r = blockIdx.x;
  if (r >= b.hdr->nreq) return;
  const BatchReq& q = b.reqs[r];
  if (b.status[r] & REQ_TOO_LARGE) {  // counts are incomplete: write nothing
    if (threadIdx.x == 0) b.nnz[r] = -1;
    return;
  }
  const long long carry = block_scan_counts<BATCH_SCAN_THREADS, 16>(b.colcnt + q.col_base, q.n, q.colptr_c, scratch,
                                                                      buf);
  if (threadIdx.x == 0) {
    if (carry <= INT_MAX) q.colptr_c[q.n] = (int)carry;
    b.nnz[r] = carry;
    if (carry > q.cap || carry > INT_MAX) atomicOr(&b.status[r], REQ_CAPACITY);
  }
}

// ---- host launchers ----
void launch_batch_plan(const BatchArgs& b, hipStream_t s) {
  k_batch_init<<<(b.max_reqs + 255) / 256 > 4 ? (b.max_reqs + 255) / 256 : 4, 256, 0, s>>>(b);
  k_batch_bounds<<<b.nblk, b.chunk < 1024 ? b.chunk : 1024, 0, s>>>(b);
  k_batch_slot_scan<<<1, 1024, 0, s>>>(b);
  k_batch_scatter<<<b.nblk, 256, 0, s>>>(b);
}

void launch_batch_scan(const BatchArgs& b, hipStream_t s) {
  k_batch_scan<<<b.max_reqs, BATCH_SCAN_THREADS, 0, s>>>(b);
}

template <bool NUM, typename V, bool BM>
static void launch_bw(int wi, const BatchArgs& b, const KArgs& a, unsigned blocks, size_t lds, hipStream_t s) {
  const int slot = BSLOT_WAVE + 2 * wi + (BM ? 1 : 0);
  const unsigned nt = 64 * PIPE_WAVES_PER_BLOCK;
  switch (wi) {
    case 0: k_batch_wave<1, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 1: k_batch_wave<2, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 2: k_batch_wave<3, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 3: k_batch_wave<4, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 4: k_batch_wave<5, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 5: k_batch_wave<6, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 6: k_batch_wave<8, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 7: k_batch_wave<10, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    case 8: k_batch_wave<12, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
    default: k_batch_wave<16, NUM, V, BM><<<blocks, nt, lds, s>>>(b, a, slot); break;
  }
}

void launch_batch_wave(int wi, bool numeric, bool f64, bool bm, const BatchArgs& b, const KArgs& a, unsigned blocks,
                       size_t lds, hipStream_t s) {
  if (!numeric) {
    if (bm) launch_bw<false, float, true>(wi, b, a, blocks, lds, s);
    else launch_bw<false, float, false>(wi, b, a, blocks, lds, s);
  } else if (f64) {
    if (bm) launch_bw<true, double, true>(wi, b, a, blocks, lds, s);
    else launch_bw<true, double, false>(wi, b, a, blocks, lds, s);
  } else {
    if (bm) launch_bw<true, float, true>(wi, b, a, blocks, lds, s);
    else launch_bw<true, float, false>(wi, b, a, blocks, lds, s);
  }
}

}  // namespace spk
