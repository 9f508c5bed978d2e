// One whole SpKAdd (plan, symbolic, numeric) with its device workspace carved from a
// given device region instead of allocated: the body of the no-allocation entry
// point.  Not part of the public ABI.
#pragma once
#include <stddef.h>

#include "spkadd.h"

namespace spk {

spkadd_status sum_in_region(void* region, size_t region_bytes, int32_t m, int32_t n, int32_t k,
                            const int32_t* const* colptr, const int32_t* const* rowidx, const void* const* values,
                            spkadd_dtype dtype, const spkadd_opts* opts, int32_t* colptr_c, int32_t* rowidx_c,
                            void* values_c, int64_t cap_c, int64_t* nnz_c, hipStream_t stream);

}  // namespace spk
