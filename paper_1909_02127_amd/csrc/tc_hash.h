// tc_hash.h - the two cuckoo hash functions of the count kernel's LDS tables.
//
// Multiplicative hashing (Knuth, TAOCP vol. 3, 6.4): the slot of key k in a half
// of 2^b slots is the top b bits of the 32-bit product k * A.  All arithmetic is
// unsigned, so the final shift is logical and the slot lies in [0, 2^b).  Ids
// below 2^24 use 24-bit operands, which map onto the full-rate v_mul_u32_u24;
// wider ids use the full 32-bit multiply.  Host-callable so the CPU tests can
// check the index range of exactly this code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

constexpr uint32_t kHashA = 0x9E3779B1u;
constexpr uint32_t kHashB = 0x7FEB352Du;
constexpr uint32_t kHashA24 = 0x9E3779u;
constexpr uint32_t kHashB24 = 0x7FEB35u;

// shift = 32 - b, 1 <= b <= 31
template <bool Wide>
__host__ __device__ __forceinline__ uint32_t hash_a(int32_t k, int shift) {
  const uint32_t x = Wide ? (uint32_t)k * kHashA : ((uint32_t)k & 0xFFFFFFu) * kHashA24;
  return x >> shift;
}
template <bool Wide>
__host__ __device__ __forceinline__ uint32_t hash_b(int32_t k, int shift) {
  const uint32_t x = Wide ? (uint32_t)k * kHashB : ((uint32_t)k & 0xFFFFFFu) * kHashB24;
  return x >> shift;
}

}  // namespace tc
