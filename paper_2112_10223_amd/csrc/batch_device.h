// Device code shared by the batched wave kernels (batch_kernels.hip: one launch per
// wave slot; batch_fused.hip: one launch per pass).
#pragma once
#include "batch_internal.h"
#include "wave_device.h"

namespace spk {

// The chunks c0, c0 + G, ... of BATCH_CHUNK list entries of one slot, for one
// wavefront.  A chunk may hold columns of several requests (they are contiguous);
// each run of one request goes through run_pipe with that request's arguments, its
// LDS layout computed here when DEV_LAYOUT (always for bitmaps: it depends on the
// request's m).  Numeric: requests whose outcome is not OK are skipped.
template <int E, bool NUM, typename V, bool BM, bool DEV_LAYOUT>
__device__ __forceinline__ void slot_chunks(const BatchArgs& b, const KArgs& a, int slot, unsigned char* base, int c0,
                                            int G) {
  const int lane = lane_id();
  const int count = b.slotoff[BSLOTS + 1 + slot];
  const int off = b.slotoff[slot];
  const int nchunks = (count + BATCH_CHUNK - 1) / BATCH_CHUNK;
  const int ts = DEV_LAYOUT ? slots_for(64 * E, 512) : a.ts_max;
  for (int c = c0; c < nchunks; c += G) {
    const int nu = min(BATCH_CHUNK, count - c * BATCH_CHUNK);
    const int g = lane < nu ? b.list[off + c * BATCH_CHUNK + lane] : 0;
    const int rl = lane < nu ? b.req_of[g] : -1;
    int pos = 0;
    while (pos < nu) {
      const int r = readlane(rl, pos);
      const uint64_t other = ballot(lane > pos && lane < nu && rl != r);
      const int end = other ? (int)__builtin_ctzll(other) : nu;
      const BatchReq& q = b.reqs[r];
      const bool skip = NUM && b.status[r] != 0;
      if (!skip) {
        KArgs ta = a;
        ta.cp = q.cp;
        ta.ri = q.ri;
        ta.va = q.va;
        ta.m = q.m;
        ta.n = q.n;
        ta.k = q.k;
        ta.colcnt = b.colcnt + q.col_base;
        ta.colptr_c = q.colptr_c;
        ta.out_r = q.out_r;
        ta.out_v = q.out_v;
        if (BM || DEV_LAYOUT) pipe_layout(E, NUM, (int)sizeof(V), ts, BM ? q.nq : 0, ta);
        // this run's columns, local to the request, in lanes 0 .. end - pos - 1
        const int src = min(lane + pos, nu - 1);
        const int ucol = __shfl(g, src) - q.col_base;
        run_pipe<E, NUM, V, BM>(ta, base, end - pos, ucol);
      }
      pos = end;
    }
  }
}

}  // namespace spk
