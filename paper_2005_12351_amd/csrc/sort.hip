// Stable device sort of (key, value) pairs on the low `bits` bits of the
// key, through rocPRIM's radix sort (hipCUB interface), for the tree build's
// larger sorts.  Kept in its own unit: its templates are slow to compile.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include "fmm_internal.h"

hipError_t dev_sort_pairs(void *tmp, size_t &tmp_bytes, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                          int32_t *vout, int n, int bits, hipStream_t s)
{
    return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0, bits, s);
}
