// Wave-bin kernels of the plain (one SpKAdd) launch.  The device code is in
// wave_device.h.
#include "wave_device.h"

namespace spk {

template <int E, bool NUM, typename V, bool BM>
__global__ __launch_bounds__(64 * PIPE_WAVES_PER_BLOCK) void k_wave_pipe(KArgs a, const int* __restrict__ list,
                                                                        int nunits) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  // Units are dealt out with stride G (all wavefronts of the launch): at any time
  // the wavefronts of one XCD (consecutive gw after the remap) work on neighbouring
  // columns, whose input rows share cache lines, instead of each wavefront walking a
  // column range of its own (too many partly used lines for the L2).
  const int G = (int)gridDim.x * PIPE_WAVES_PER_BLOCK;
  const int gw = xcd_remap(blockIdx.x, gridDim.x) * PIPE_WAVES_PER_BLOCK + w;
  if (gw >= nunits) return;  // no block-wide barriers in this kernel
  const int nu = (nunits - gw + G - 1) / G;  // <= upw <= 64
  const int ucol = lane < nu ? list[gw + lane * G] : 0;
  run_pipe<E, NUM, V, BM>(a, smem + w * a.slice_bytes, nu, ucol);
}

// ---- host side ----
bool wave_pipe_ok(int k, int alpha_num_q) { return k <= 64 && alpha_num_q == 512; }

void lds_layout_pipe(int bin, bool numeric, int vbytes, int ts_max, int bm_nq, KArgs& a) {
  pipe_layout(wave_bin_E(bin), numeric, vbytes, ts_max, bm_nq, a);
}

template <int E, bool NUM, typename V>
static void launch_pipe_e(const KArgs& a, const int* list, int n, unsigned blocks, size_t lds, hipStream_t s) {
  if (a.bm_nq > 0)
    k_wave_pipe<E, NUM, V, true><<<blocks, 64 * PIPE_WAVES_PER_BLOCK, lds, s>>>(a, list, n);
  else
    k_wave_pipe<E, NUM, V, false><<<blocks, 64 * PIPE_WAVES_PER_BLOCK, lds, s>>>(a, list, n);
}

template <bool NUM, typename V>
static hipError_t launch_pipe_t(int bin, const KArgs& a, const int* list, int n, hipStream_t s) {
  const int waves = (n + a.upw - 1) / a.upw;
  const unsigned blocks = (unsigned)((waves + PIPE_WAVES_PER_BLOCK - 1) / PIPE_WAVES_PER_BLOCK);
  const size_t lds = (size_t)a.slice_bytes * PIPE_WAVES_PER_BLOCK;
  switch (bin) {
    case BIN_W1: launch_pipe_e<1, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W2: launch_pipe_e<2, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W3: launch_pipe_e<3, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W4: launch_pipe_e<4, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W5: launch_pipe_e<5, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W6: launch_pipe_e<6, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W8: launch_pipe_e<8, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W10: launch_pipe_e<10, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W12: launch_pipe_e<12, NUM, V>(a, list, n, blocks, lds, s); break;
    case BIN_W16: launch_pipe_e<16, NUM, V>(a, list, n, blocks, lds, s); break;
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
