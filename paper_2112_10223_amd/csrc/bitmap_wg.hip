// Workgroup bitmap accumulator for row windows (Section III-B, Algorithms 7-8) and
// workgroup columns whose row range is narrow enough: one bit per row of the unit's
// range [rlo, rhi) in LDS.  Symbolic (Algorithm 6): an OR that finds its bit clear
// counts a new row.  Numeric (Algorithm 5): OR with return marks each row's first
// entry, a block-wide popcount prefix over groups of words gives rank(row) = the row's
// position in the sorted output, the first entry stores (row, value) at its rank in
// an LDS staging area and later entries add by compare-and-swap; the unit is then
// written out coalesced.  No hash table and no sort: the bitmap is the "partitioned
// SPA" the paper proposes for row-partitioned accumulation, with a rank in place of a
// dense value array.
//
// A unit wider than a.wg_span_max rows is left to the hash kernel (k_hash_wg skips the
// units this kernel takes, so both can run over one unit list).
#include "bitmap_wg_device.h"

namespace spk {

template <int NT, int EW, bool NUM, bool WIN, typename V, int G>
__global__ __launch_bounds__(NT) void k_bitmap_wg(KArgs a, const int* __restrict__ list, int nunits) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long red[NT / 64 + 1];
  __shared__ int info;
  const int unit = xcd_remap(blockIdx.x, gridDim.x);
  if (unit >= nunits) return;  // uniform over the block
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
  bitmap_wg_unit<NT, EW, NUM, WIN, V, G>(a, smem, red, &info, unit, j, blo, rlo, rhi);
}

// ---- host side ----

// 2^18 rows: 32 KiB of bitmap and 4 KiB of prefix (groups of four words), with the
// staging area over the bitmap four numeric workgroups per CU (measured on R-MAT
// windows: 2^17 leaves more windows to the hash kernel, 2^19 halves the resident
// workgroups; both slower).
int bitmap_wg_span_max() { return 1 << 18; }

int bitmap_wg_regs(int bin) { return (bin == BIN_G1 ? G1_THREADS : G2_THREADS) * 8; }

// Bitmap words [0, off_pre), the group prefix after them (numeric only), then the
// staging area of `cap` output entries.  The staging area overlays the bitmap when
// that is safe: a unit whose entries all sit in registers (u <= one_max) has read
// every rank before it stages; a unit with more entries (a window, then at most cap
// rows wide: refinement only stops splitting a window that holds more than cap
// entries once it is that narrow) keeps its bitmap below `cap` rows' worth of words
// and its prefix words at off_pre, so its staging area goes between the two.
void lds_layout_bitmap_wg(bool numeric, int vbytes, int k, int span_max, int cap, int one_max, bool all_one, int G,
                          KArgs& a) {
  auto align16 = [](int x) { return (x + 15) & ~15; };
  const int ngrp = (span_max + 32 * G - 1) / (32 * G);
  a.off_bm = 0;
  a.off_pre = align16(ngrp * G * 4);  // bitmap words
  a.wg_group = G;
  int off = a.off_pre;
  a.wg_overlay = 0;
  if (numeric) {
    const int pw_end = align16(a.off_pre + ngrp * 2);
    const int vstage = align16(cap * vbytes), stage = vstage + align16(cap * 4);
    const int below = align16((cap + 32 * G - 1) / (32 * G) * G * 4);  // bitmap of a unit at most cap rows wide
    if (all_one) {
      a.wg_overlay = 1;
      a.off_bvals = 0;
      off = pw_end > stage ? pw_end : stage;
    } else if (cap <= one_max && below + stage <= a.off_pre) {
      a.wg_overlay = 1;
      a.off_bvals = below;
      off = pw_end;
    } else {
      a.off_bvals = pw_end;
      off = pw_end + stage;
    }
    a.off_brows = a.off_bvals + vstage;
  } else {
    a.off_bvals = a.off_brows = 0;
  }
  a.off_P = off;
  off = (off + (k + 1) * 4 + 7) & ~7;
  a.off_adj = off;
  off += k * 8;
  a.off_adjv = off;
  if (numeric) off += k * 8;
  off = align16(off);
  a.off_mark = off;  // segment-start mask of the units whose entries fit registers
  off += seg_mask_bytes(k);
  a.slice_bytes = align16(off);
  a.wg_span_max = span_max;
  a.wg_cap = cap;
}

template <bool NUM, typename V, int G>
static hipError_t launch_bw(int bin, const KArgs& a, const int* list, int n, hipStream_t s) {
  const size_t lds = (size_t)a.slice_bytes;
  constexpr int EW = 8;  // 4096 (G2, windows) or 2048 (G1) entries in registers: at least cap_in
  if (bin == BIN_WIN)
    k_bitmap_wg<G2_THREADS, EW, NUM, true, V, G><<<n, G2_THREADS, lds, s>>>(a, list, n);
  else if (bin == BIN_G1)
    k_bitmap_wg<G1_THREADS, EW, NUM, false, V, G><<<n, G1_THREADS, lds, s>>>(a, list, n);
  else
    k_bitmap_wg<G2_THREADS, EW, NUM, false, V, G><<<n, G2_THREADS, lds, s>>>(a, list, n);
  return hipGetLastError();
}

hipError_t launch_bitmap_wg(int bin, bool numeric, bool f64, const KArgs& a, const int* d_list, int nunits,
                            hipStream_t s) {
  if (nunits <= 0) return hipSuccess;
  if (bin != BIN_G1 && bin != BIN_G2 && bin != BIN_WIN) return hipErrorInvalidValue;
  if (!numeric) return launch_bw<false, float, 2>(bin, a, d_list, nunits, s);  // (no prefix)
  if (a.wg_group == 4)
    return f64 ? launch_bw<true, double, 4>(bin, a, d_list, nunits, s) : launch_bw<true, float, 4>(bin, a, d_list, nunits, s);
  return f64 ? launch_bw<true, double, 2>(bin, a, d_list, nunits, s) : launch_bw<true, float, 2>(bin, a, d_list, nunits, s);
}

}  // namespace spk
