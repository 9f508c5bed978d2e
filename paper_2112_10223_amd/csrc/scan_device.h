// Exclusive scan of int32 counts by one workgroup (colptr of an output from its
// column counts).
#pragma once
#include <climits>

#include "device.h"

namespace spk {

// out[x] = in[0] + ... + in[x-1] for x in [0, n); returns the total.  Tiles of NT*PER
// entries pass through `buf` (NT*PER ints of LDS): loads and stores are coalesced
// (consecutive lanes, consecutive entries; the load index is clamped instead of
// guarded so that all of a thread's loads are in flight together), and each thread
// scans PER consecutive entries of the tile.  Prefixes above INT_MAX are written
// truncated; the caller reports the overflow from the total.  `scratch` holds
// NT/64 + 1 values; every thread of the block must call this.
template <int NT, int PER>
__device__ __forceinline__ long long block_scan_counts(const int* __restrict__ in, int n, int* __restrict__ out,
                                                       long long* scratch, int* buf) {
  long long carry = 0;
  for (int tile = 0; tile < n; tile += NT * PER) {
    const int len = min(n - tile, NT * PER);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = q * NT + (int)threadIdx.x;
      const int v = in[tile + min(x, len - 1)];
      buf[x] = x < len ? v : 0;
    }
    __syncthreads();
    int v[PER];
    long long s = 0;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      v[t] = buf[threadIdx.x * PER + t];
      s += v[t];
    }
    long long chunk = 0;
    // (its barriers also order every read of buf above before the writes below)
    long long run = carry + block_excl_scan<NT>(s, scratch, &chunk);
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      buf[threadIdx.x * PER + t] = (int)run;
      run += v[t];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = q * NT + (int)threadIdx.x;
      if (x < len) out[tile + x] = buf[x];
    }
    __syncthreads();  // buf is reloaded by the next tile
    carry += chunk;
  }
  return carry;
}

}  // namespace spk
