// tc_hash.h - the two cuckoo hash functions of the count kernel's LDS tables.
//
// Multiplicative hashing (Knuth, TAOCP vol. 3, 6.4): the slot of key k in a half
// of 2^b slots is the top b bits of the 32-bit product x * A.  All arithmetic is
// unsigned, so the final shift is logical and the slot lies in [0, 2^b).  The
// operands are 24-bit, which maps onto the full-rate v_mul_u32_u24; ids of 2^24
// and above are first folded to 24 bits.  Host-callable so the CPU tests can
// check the index range of exactly this code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

constexpr uint32_t kHashA24 = 0x9E3779u;
constexpr uint32_t kHashB24 = 0x7FEB35u;

// The 24-bit multiplier input for a key.  Ids below 2^24 are used as they are;
// wider ids fold their top bits into the low 24 (two VALU ops, shared by both
// hashes), which keeps both hashes on the full-rate multiplier.
template <bool Wide>
__host__ __device__ __forceinline__ uint32_t hash_input(int32_t k) {
  return Wide ? ((uint32_t)k ^ ((uint32_t)k >> 24)) : (uint32_t)k;
}

// shift = 32 - b, 1 <= b <= 31; x = hash_input<Wide>(k)
__host__ __device__ __forceinline__ uint32_t hash_a_of(uint32_t x, int shift) {
  return ((x & 0xFFFFFFu) * kHashA24) >> shift;
}
__host__ __device__ __forceinline__ uint32_t hash_b_of(uint32_t x, int shift) {
  return ((x & 0xFFFFFFu) * kHashB24) >> shift;
}
template <bool Wide>
__host__ __device__ __forceinline__ uint32_t hash_a(int32_t k, int shift) {
  return hash_a_of(hash_input<Wide>(k), shift);
}
template <bool Wide>
__host__ __device__ __forceinline__ uint32_t hash_b(int32_t k, int shift) {
  return hash_b_of(hash_input<Wide>(k), shift);
}

}  // namespace tc
