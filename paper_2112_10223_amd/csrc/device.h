// Wavefront and workgroup primitives for gfx950 (64-lane wavefronts).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace spk {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders this wavefront's LDS accesses before / after the point for the compiler.
// The hardware already executes one wavefront's LDS instructions in order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of mask below this lane.
__device__ __forceinline__ int mbcnt(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---- DPP (data-parallel primitives) wave scans for 32-bit integers ----
// update_dpp(old, src, ctrl, row_mask, bank_mask, bound_ctrl=false): lanes whose
// source is outside the row, or whose row is masked off, keep `old`.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ int dpp_i32(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWMASK, 0xf, false);
}

// Inclusive add-scan over the 64 lanes: row_shr 1,2,4,8 inside each row of 16, then
// row_bcast:15 and row_bcast:31 carry the row totals (GFX9 DPP).
__device__ __forceinline__ int wave_scan_add(int x) {
  x += dpp_i32<0x111>(0, x);
  x += dpp_i32<0x112>(0, x);
  x += dpp_i32<0x114>(0, x);
  x += dpp_i32<0x118>(0, x);
  x += dpp_i32<0x142, 0xa>(0, x);
  x += dpp_i32<0x143, 0xc>(0, x);
  return x;
}

__device__ __forceinline__ int wave_scan_max(int x) {
  const int lo = -2147483647 - 1;
  x = max(x, dpp_i32<0x111>(lo, x));
  x = max(x, dpp_i32<0x112>(lo, x));
  x = max(x, dpp_i32<0x114>(lo, x));
  x = max(x, dpp_i32<0x118>(lo, x));
  x = max(x, dpp_i32<0x142, 0xa>(lo, x));
  x = max(x, dpp_i32<0x143, 0xc>(lo, x));
  return x;
}

__device__ __forceinline__ int wave_scan_min(int x) {
  const int hi = 2147483647;
  x = min(x, dpp_i32<0x111>(hi, x));
  x = min(x, dpp_i32<0x112>(hi, x));
  x = min(x, dpp_i32<0x114>(hi, x));
  x = min(x, dpp_i32<0x118>(hi, x));
  x = min(x, dpp_i32<0x142, 0xa>(hi, x));
  x = min(x, dpp_i32<0x143, 0xc>(hi, x));
  return x;
}

__device__ __forceinline__ int readlane(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }
__device__ __forceinline__ int wave_total_add(int x) { return readlane(wave_scan_add(x), 63); }
__device__ __forceinline__ int wave_total_max(int x) { return readlane(wave_scan_max(x), 63); }
__device__ __forceinline__ int wave_total_min(int x) { return readlane(wave_scan_min(x), 63); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  if constexpr (std::is_same<T, int>::value) return wave_scan_add(x);
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
  if constexpr (std::is_same<T, int>::value) return wave_total_add(x);
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    T y = __shfl_xor(x, d, 64);
    x = y < x ? y : x;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_bcast(T x, int src) {
  return __shfl(x, src, 64);
}

// Exclusive scan over the NT threads of a block.  `scratch` holds NT/64 + 1 values.
// Contains two __syncthreads; every thread of the block must call it.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* scratch, T* total = nullptr) {
  constexpr int NW = NT / 64;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  T incl = wave_incl_scan(x);
  if (lane == 63) scratch[w] = incl;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    T s = scratch[v];
    before += v < w ? s : T(0);
    all += s;
  }
  if (total) *total = all;
  __syncthreads();
  return before + incl - x;
}

template <int NT, typename T>
__device__ __forceinline__ T block_sum(T x, T* scratch) {
  constexpr int NW = NT / 64;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  T s = wave_sum(x);
  if (lane == 0) scratch[w] = s;
  __syncthreads();
  T all = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) all += scratch[v];
  __syncthreads();
  return all;
}

// Blocks are handed to the 8 XCDs of the device round-robin (block b runs on XCD
// b % 8).  This remaps the hardware block id so that each XCD gets a contiguous run
// of logical blocks, which keeps neighbouring columns in one XCD's L2.
// Loads and stores through a 64-bit address known to be global memory (not a
// generic pointer: generic accesses share the LDS wait counter).
template <typename T>
__device__ __forceinline__ T gload(long long addr) {
  return *(const __attribute__((address_space(1))) T*)addr;
}

template <typename T>
__device__ __forceinline__ void gstore(long long addr, T v) {
  *(__attribute__((address_space(1))) T*)addr = v;
}

// A store that is not read again by this kernel (the output of a numeric pass): the
// nontemporal hint keeps the written lines from displacing input lines that a
// neighbouring column is about to read from the L2.
template <typename T>
__device__ __forceinline__ void gstore_nt(long long addr, T v) {
  __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)addr);
}

// A wave-uniform 64-bit value moved into scalar registers (lane 0's copy).  The
// builtin returns int: each half goes through unsigned so it is not sign-extended.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long x) {
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x >> 32));
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
  return ((unsigned long long)hi << 32) | (unsigned long long)lo;
}

__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int x = b & 7, q = b >> 3;
  const int per = G >> 3, rem = G & 7;
  return x * per + (x < rem ? x : rem) + q;
}

__device__ __forceinline__ int ceil_log2(int v) {  // v >= 1
  return v <= 1 ? 0 : 32 - __clz(v - 1);
}

}  // namespace spk
