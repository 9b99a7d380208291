// Device-wide primitives from hipCUB: the exclusive scans of the extraction's 0/1 flags, and
// for the explicit reduced camera system a stable radix sort of (32-bit key, 64-bit value)
// pairs and an exclusive prefix sum. Kept in a translation unit of their own so that the
// library headers stay out of the kernel file.
#include "ba_kernels.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>

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

namespace {

// Flag i of the scan input: 1 for a set flag, 0 beyond the last element (index n), so that an
// exclusive scan over n + 1 items writes the total at out[n].
struct FlagU8 {
  const uint8_t* a;
  int64_t n;
  __host__ __device__ int operator()(int64_t i) const { return i < n && a[i] != 0 ? 1 : 0; }
};
struct FlagCM {
  const uint8_t* vrow_cm;
  const int* cm_cam;
  const uint8_t* fixed;
  int64_t n;
  __host__ __device__ int operator()(int64_t i) const {
    return i < n && vrow_cm[i] != 0 && !fixed[cm_cam[i]] ? 1 : 0;
  }
};

template <class F>
using FlagIter = hipcub::TransformInputIterator<int, F, hipcub::CountingInputIterator<int64_t>>;

template <class F>
hipError_t flag_scan(hipStream_t s, int64_t n, F f, int* out, void* temp, size_t temp_bytes) {
  if (n < 0 || n + 1 > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  FlagIter<F> in(hipcub::CountingInputIterator<int64_t>(0), f);
  return hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, in, out, int(n + 1), s);
}

}  // namespace

size_t scan_temp_bytes(int64_t n) {
  size_t a = 0, b = 0;
  FlagIter<FlagU8> iu(hipcub::CountingInputIterator<int64_t>(0), FlagU8{nullptr, n});
  FlagIter<FlagCM> ic(hipcub::CountingInputIterator<int64_t>(0), FlagCM{nullptr, nullptr, nullptr, n});
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, a, iu, (int*)nullptr, int(n + 1));
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b, ic, (int*)nullptr, int(n + 1));
  return std::max(a, b);
}

hipError_t launch_scan_u8(hipStream_t s, int64_t n, const uint8_t* flags, int* out, void* temp,
                          size_t temp_bytes) {
  return flag_scan(s, n, FlagU8{flags, n}, out, temp, temp_bytes);
}

hipError_t launch_scan_cm(hipStream_t s, int64_t n, const uint8_t* vrow_cm, const int* cm_cam,
                          const uint8_t* fixed, int* out, void* temp, size_t temp_bytes) {
  return flag_scan(s, n, FlagCM{vrow_cm, cm_cam, fixed, n}, out, temp, temp_bytes);
}

}  // namespace iba
