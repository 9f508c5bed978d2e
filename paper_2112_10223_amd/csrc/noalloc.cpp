// spkadd_sum_noalloc: the whole SpKAdd in one call, with every byte of device
// workspace in a file-scope device array instead of an allocation.
//
// Host code may not pass `scratch` itself to a kernel or a copy (in host code the
// name stands for a host-side shadow, not a device address).  The device address of
// each GPU's copy is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"
#include "region.h"
#include "spkadd.h"

namespace {

__device__ __align__(256) unsigned char scratch[SPKADD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` on each device
std::mutex g_mu;

// The address of the current device's copy of `scratch` (looked up on first use,
// with that device current).
spkadd_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return spk::report_error(SPKADD_ERR_HIP, "hipGetDevice failed");
  }
  if (dev < 0 || dev >= kMaxDevices) return spk::report_error(SPKADD_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return spk::report_error(SPKADD_ERR_HIP, "hipGetSymbolAddress of the scratch array failed");
    }
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return SPKADD_OK;
}

}  // namespace

extern "C" spkadd_status spkadd_sum_noalloc(int32_t m, int32_t n, int32_t k, const int32_t* const* colptr,
                                            const int32_t* const* rowidx, const void* const* values,
                                            spkadd_dtype dtype, const spkadd_opts* opts, int32_t* colptr_c,
                                            int32_t* rowidx_c, void* values_c, int64_t cap_c, int64_t* nnz_c,
                                            hipStream_t stream) {
  void* region = nullptr;
  const spkadd_status st = scratch_address(&region);
  if (st != SPKADD_OK) return st;
  return spk::sum_in_region(region, (size_t)SPKADD_NOALLOC_SCRATCH_BYTES, m, n, k, colptr, rowidx, values, dtype,
                            opts, colptr_c, rowidx_c, values_c, cap_c, nnz_c, stream);
}
