// Device-wide primitives of the explicit reduced camera system, from hipCUB: a stable radix
// sort of (32-bit key, 64-bit value) pairs and an exclusive prefix sum. Kept in a translation
// unit of their own so that the library headers stay out of the kernel file.
#include "ba_kernels.h"

#include <hipcub/hipcub.hpp>

namespace iba {

size_t sort_pairs64_temp_bytes(int n, int end_bit) {
  size_t bytes = 0;
  const uint32_t* k = nullptr;
  const uint64_t* v = nullptr;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, k, (uint32_t*)nullptr, v,
                                           (uint64_t*)nullptr, n, 0, end_bit);
  return bytes;
}

hipError_t sort_pairs64(void* temp, size_t temp_bytes, const uint32_t* keys_in,
                        uint32_t* keys_out, const uint64_t* vals_in, uint64_t* vals_out, int n,
                        int end_bit, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys_in, keys_out, vals_in,
                                            vals_out, n, 0, end_bit, s);
}

size_t exclusive_sum_temp_bytes(int n) {
  size_t bytes = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int64_t*)nullptr,
                                         (int64_t*)nullptr, n);
  return bytes;
}

hipError_t exclusive_sum(void* temp, size_t temp_bytes, const int64_t* in, int64_t* out, int n,
                         hipStream_t s) {
  return hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, in, out, n, s);
}

}  // namespace iba
