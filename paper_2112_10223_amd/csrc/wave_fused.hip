// Symbolic pass of all wave bins in one persistent launch (Algorithm 6 per column,
// with the bins of Section III-A).  The launch needs no bin count on the host, so
// the plan does not wait for the device before the symbolic pass starts.
#include "wave_device.h"
#include "wave_fused.h"

namespace spk {

// Units c0, c0 + G, ... of one bin for one wavefront, in rounds of at most 64 (a
// wavefront's pipeline holds the column ids of a round in its lanes).
template <int E, bool BM>
__device__ __forceinline__ void sym_bin(const KArgs& a0, const WaveBinTable& t, int wi, const int* __restrict__ list,
                                        int cnt, int c0, int G, unsigned char* base) {
  KArgs a = a0;
  pipe_layout(E, false, 4, t.ts[wi], BM ? t.bm_nq[wi] : 0, a);
  const int lane = lane_id();
  for (long long first = c0; first < cnt; first += 64LL * G) {
    const int nu = (int)((cnt - first + G - 1) / G < 64 ? (cnt - first + G - 1) / G : 64);
    const int ucol = lane < nu ? list[first + (long long)lane * G] : 0;
    run_pipe<E, false, float, BM>(a, base, nu, ucol);
  }
}

template <int E>
__device__ __forceinline__ void sym_bin_any(const KArgs& a, const WaveBinTable& t, int wi,
                                            const int* __restrict__ list, int cnt, int c0, int G,
                                            unsigned char* base) {
  if (t.bm_nq[wi] > 0) sym_bin<E, true>(a, t, wi, list, cnt, c0, G, base);
  else sym_bin<E, false>(a, t, wi, list, cnt, c0, G, base);
}

// The units of all wave bins form one sequence, longest columns first; wavefront gw
// of G takes units gw, gw + G, ... of that sequence.
__global__ __launch_bounds__(64 * PIPE_WAVES_PER_BLOCK) void k_wave_sym_fused(KArgs a, WaveBinTable t,
                                                                             const int* __restrict__ list,
                                                                             const int* __restrict__ binoff) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = threadIdx.x >> 6;
  const int G = (int)gridDim.x * PIPE_WAVES_PER_BLOCK;
  const int gw = xcd_remap(blockIdx.x, gridDim.x) * PIPE_WAVES_PER_BLOCK + w;
  unsigned char* base = smem + w * a.slice_bytes;
  long long before = 0;  // units of the bins already passed
  for (int wi = NWAVE_BINS - 1; wi >= 0; --wi) {
    const int b = BIN_W1 + wi;
    const int off = binoff[b], cnt = binoff[b + 1] - off;
    if (cnt <= 0) continue;
    // first unit c of this bin with (before + c) == gw (mod G)
    const int c0 = (int)(((long long)gw - before % G + G) % G);
    before += cnt;
    if (c0 >= cnt) continue;
    const int* bl = list + off;
    switch (wi) {
      case 0: sym_bin_any<1>(a, t, wi, bl, cnt, c0, G, base); break;
      case 1: sym_bin_any<2>(a, t, wi, bl, cnt, c0, G, base); break;
      case 2: sym_bin_any<3>(a, t, wi, bl, cnt, c0, G, base); break;
      case 3: sym_bin_any<4>(a, t, wi, bl, cnt, c0, G, base); break;
      case 4: sym_bin_any<5>(a, t, wi, bl, cnt, c0, G, base); break;
      case 5: sym_bin_any<6>(a, t, wi, bl, cnt, c0, G, base); break;
      case 6: sym_bin_any<8>(a, t, wi, bl, cnt, c0, G, base); break;
      case 7: sym_bin_any<10>(a, t, wi, bl, cnt, c0, G, base); break;
      case 8: sym_bin_any<12>(a, t, wi, bl, cnt, c0, G, base); break;
      default: sym_bin_any<16>(a, t, wi, bl, cnt, c0, G, base); break;
    }
  }
}

hipError_t launch_wave_sym_fused(const KArgs& a, const WaveBinTable& t, const int* d_list, const int* d_binoff,
                                 unsigned blocks, hipStream_t s) {
  const size_t lds = (size_t)a.slice_bytes * PIPE_WAVES_PER_BLOCK;
  k_wave_sym_fused<<<blocks, 64 * PIPE_WAVES_PER_BLOCK, lds, s>>>(a, t, d_list, d_binoff);
  return hipGetLastError();
}

}  // namespace spk
