// Ordered values (ordered.hip), the pass behind SPKADD_FLAG_ORDERED.  Not part of
// the public ABI.
#pragma once
#include "internal.h"

namespace spk {

// Every output entry of the listed columns (and of the row windows when nwin > 0)
// summed again in input order.  cap bounds the output entries of one unit; the LDS
// one unit needs is ordered_lds_bytes(k, cap, vbytes).
int ordered_lds_bytes(int k, int cap, int vbytes);
hipError_t launch_ordered(const KArgs& a, const int* d_cols, int ncols, int nwin, int cap, bool f64, int n_cu,
                          hipStream_t s);

}  // namespace spk
