// The fused batched launch (include/spkadd_batch.h): each pass (symbolic, numeric)
// of a run in one persistent kernel over every wave slot.  Against one launch per
// slot it saves the launches and the per-slot tails (the waves of a slot kernel wait
// for its slowest chunk) at the price of the largest slot's registers and LDS.
#include "batch_device.h"
#include "bitmap_wg_device.h"

namespace spk {

template <bool NUM, typename V>
__device__ __forceinline__ void fused_slot(int wi, int bm, const BatchArgs& b, const KArgs& a, int slot,
                                           unsigned char* base, int c0, int G) {
#define SPK_FUSED_CASE(I, E)                                                    \
  case I:                                                                       \
    if (bm) slot_chunks<E, NUM, V, true, true>(b, a, slot, base, c0, G);        \
    else slot_chunks<E, NUM, V, false, true>(b, a, slot, base, c0, G);          \
    break;
  switch (wi) {
    SPK_FUSED_CASE(0, 1)
    SPK_FUSED_CASE(1, 2)
    SPK_FUSED_CASE(2, 3)
    SPK_FUSED_CASE(3, 4)
    SPK_FUSED_CASE(4, 5)
    SPK_FUSED_CASE(5, 6)
    SPK_FUSED_CASE(6, 8)
    SPK_FUSED_CASE(7, 10)
    SPK_FUSED_CASE(8, 12)
    default:
      if (bm) slot_chunks<16, NUM, V, true, true>(b, a, slot, base, c0, G);
      else slot_chunks<16, NUM, V, false, true>(b, a, slot, base, c0, G);
      break;
  }
#undef SPK_FUSED_CASE
}

// Persistent, one launch per pass for every wave slot.  The chunks of
// all slots form one sequence, longest columns first; wavefront gw of G takes chunks
// gw, gw + G, ... of that sequence.  The LDS slice is the largest any slot needs.
template <bool NUM, typename V>
__global__ __launch_bounds__(64 * PIPE_WAVES_PER_BLOCK) void k_batch_fused(BatchArgs b, KArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = threadIdx.x >> 6;
  const int G = (int)gridDim.x * PIPE_WAVES_PER_BLOCK;
  const int gw = xcd_remap(blockIdx.x, gridDim.x) * PIPE_WAVES_PER_BLOCK + w;
  unsigned char* base = smem + w * a.slice_bytes;
  int before = 0;  // chunks of the slots already passed
  for (int wi = NWAVE_BINS - 1; wi >= 0; --wi) {
    for (int bm = 0; bm < 2; ++bm) {
      const int slot = BSLOT_WAVE + 2 * wi + bm;
      const int nchunks = (b.slotoff[BSLOTS + 1 + slot] + BATCH_CHUNK - 1) / BATCH_CHUNK;
      if (nchunks == 0) continue;
      // first chunk c of this slot with (before + c) == gw (mod G)
      const int c0 = (int)(((long long)gw - before % G + G) % G);
      if (c0 < nchunks) fused_slot<NUM, V>(wi, bm, b, a, slot, base, c0, G);
      before += nchunks;
    }
  }
}

// Persistent, one launch per pass: workgroup w of W takes the columns w, w + W, ...
// of the workgroup slot, each through the workgroup bitmap over its request's rows.
template <int THREADS, bool NUM, typename V>
__global__ __launch_bounds__(THREADS) void k_batch_wg(BatchArgs b, KArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long red[THREADS / 64 + 1];
  __shared__ int info;
  const int count = b.slotoff[BSLOTS + 1 + BSLOT_WG];
  const int off = b.slotoff[BSLOT_WG];
  for (int item = xcd_remap(blockIdx.x, gridDim.x); item < count; item += gridDim.x) {
    const int g = b.list[off + item];
    const int r = b.req_of[g];
    const BatchReq& q = b.reqs[r];
    if (NUM && b.status[r] != 0) continue;  // uniform: the request's outcome is not OK
    KArgs ta = a;
    ta.cp = q.cp;
    ta.ri = q.ri;
    ta.va = q.va;
    ta.m = q.m;
    ta.n = q.n;
    ta.k = q.k;
    int ktop = 0;  // largest power of two <= k - 1
    while ((ktop << 1) <= q.k - 1) ktop = ktop ? ktop << 1 : 1;
    ta.ktop = q.k > 1 ? ktop : 0;
    ta.colcnt = b.colcnt + q.col_base;
    ta.colptr_c = q.colptr_c;
    ta.out_r = q.out_r;
    ta.out_v = q.out_v;
    bitmap_wg_unit<THREADS, BATCH_WG_U / THREADS, NUM, false, V>(ta, smem, red, &info, 0, g - q.col_base, 0, 0,
                                                                q.m);
    __syncthreads();  // the next column rewrites the LDS this one may still read
  }
}

template <int THREADS>
static void launch_wg_t(bool numeric, bool f64, const BatchArgs& b, const KArgs& a, unsigned blocks, hipStream_t s) {
  const size_t lds = (size_t)a.slice_bytes;
  if (!numeric) k_batch_wg<THREADS, false, float><<<blocks, THREADS, lds, s>>>(b, a);
  else if (f64) k_batch_wg<THREADS, true, double><<<blocks, THREADS, lds, s>>>(b, a);
  else k_batch_wg<THREADS, true, float><<<blocks, THREADS, lds, s>>>(b, a);
}

void launch_batch_wg(bool numeric, bool f64, int threads, const BatchArgs& b, const KArgs& a, unsigned blocks,
                     hipStream_t s) {
  if (threads == 512) launch_wg_t<512>(numeric, f64, b, a, blocks, s);
  else launch_wg_t<256>(numeric, f64, b, a, blocks, s);
}

int batch_fused_blocks_per_cu(bool numeric, bool f64, size_t lds) {
  const int nt = 64 * PIPE_WAVES_PER_BLOCK;
  int blocks = 0;
  hipError_t e;
  if (!numeric) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_fused<false, float>, nt, lds);
  else if (f64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_fused<true, double>, nt, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_fused<true, float>, nt, lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return blocks;
}

void launch_batch_fused(bool numeric, bool f64, const BatchArgs& b, const KArgs& a, unsigned blocks, size_t lds,
                        hipStream_t s) {
  const unsigned nt = 64 * PIPE_WAVES_PER_BLOCK;
  if (!numeric) k_batch_fused<false, float><<<blocks, nt, lds, s>>>(b, a);
  else if (f64) k_batch_fused<true, double><<<blocks, nt, lds, s>>>(b, a);
  else k_batch_fused<true, float><<<blocks, nt, lds, s>>>(b, a);
}

}  // namespace spk
