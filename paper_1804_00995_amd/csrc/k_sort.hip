// k_sort.hip -- radix sort of (64-bit key, 32-bit value) pairs, used to put the near and far
// block lists in their defined order.  The keys are unique, so the result is fully determined.
#include <rocprim/device/device_radix_sort.hpp>

#include "hmx_host.h"

namespace hmx {

void radix_sort_u64_pairs(const uint64_t* kin, uint64_t* kout, const int32_t* vin, int32_t* vout,
                          int64_t n, int end_bit, DevBuf<unsigned char>& tmp, hipStream_t s) {
  if (n <= 0) return;
  size_t bytes = 0;
  HMX_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0u,
                                    (unsigned)end_bit, s));
  tmp.alloc(std::max<size_t>(bytes, 1));
  HMX_HIP(rocprim::radix_sort_pairs((void*)tmp.p, bytes, kin, kout, vin, vout, (size_t)n, 0u,
                                    (unsigned)end_bit, s));
}

}  // namespace hmx
