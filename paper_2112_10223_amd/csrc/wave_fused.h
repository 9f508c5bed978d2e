// The symbolic pass of every wave bin in one launch (wave_fused.hip).  Not part of
// the public ABI.
#pragma once
#include "internal.h"

namespace spk {

// Per wave bin (index bin - BIN_W1): bitmap rows of 256 words (0: hash tables) and
// symbolic table slots; the kernel derives each bin's LDS layout from them.
struct WaveBinTable {
  int bm_nq[NWAVE_BINS];
  int ts[NWAVE_BINS];
};

// Counts the distinct rows of every column of the wave bins.  The bins' column
// lists and offsets are read on the device (d_list, d_binoff as the binning kernels
// leave them), so the host needs no bin count to launch it.  a.slice_bytes is the
// largest slice of any wave bin; blocks is the grid (resident blocks of four
// wavefronts).
hipError_t launch_wave_sym_fused(const KArgs& a, const WaveBinTable& t, const int* d_list, const int* d_binoff,
                                 unsigned blocks, hipStream_t s);

}  // namespace spk
