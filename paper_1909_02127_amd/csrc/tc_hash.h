// tc_hash.h - the two cuckoo hash functions of the count kernel's LDS tables.
//
// Multiplicative hashing (Knuth, TAOCP vol. 3, 6.4) with one product per key:
// p = x * A over 24-bit operands (the full-rate v_mul_u32_u24), the slot in half
// a is the top b bits of p and the slot in half b the b bits just below them
// (b <= 16).  Two bit fields of one multiply-shift hash act as the pair of
// cuckoo hashes; for ids packed in a window a few times the key count (the
// small graphs of a batch) they place far fewer keys in the stash than two
// products with different multipliers, whose slot pairs for nearby ids fall on
// a lattice.  All arithmetic is unsigned, so shifts are logical and slots lie
// in [0, 2^b).  Ids of 2^24 and above are first folded to 24 bits.
// Host-callable so the CPU tests can check the index range of exactly this
// code; the device probes take slot b with one bit-field extract.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

constexpr uint32_t kHashA24 = 0x9E3779u;

// The 24-bit multiplier input for a key.  Ids below 2^24 are used as they are;
// wider ids fold their top bits into the low 24 (two VALU ops).
template <bool Wide>
__host__ __device__ __forceinline__ uint32_t hash_input(int32_t k) {
  return Wide ? ((uint32_t)k ^ ((uint32_t)k >> 24)) : (uint32_t)k;
}

__host__ __device__ __forceinline__ uint32_t hash_product(uint32_t x) {
  return (x & 0xFFFFFFu) * kHashA24;
}

// shift = 32 - b, 1 <= b <= 16; p = hash_product(x)
__host__ __device__ __forceinline__ uint32_t slot_a_of(uint32_t p, int shift) {
  return p >> shift;
}
__host__ __device__ __forceinline__ uint32_t slot_b_of(uint32_t p, int shift) {
  const uint32_t b = 32u - (uint32_t)shift;
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_ubfe(p, 32u - 2u * b, b);
#else
  return (p >> (32u - 2u * b)) & ((1u << b) - 1u);
#endif
}

// x = hash_input<Wide>(k)
__host__ __device__ __forceinline__ uint32_t hash_a_of(uint32_t x, int shift) {
  return slot_a_of(hash_product(x), shift);
}
__host__ __device__ __forceinline__ uint32_t hash_b_of(uint32_t x, int shift) {
  return slot_b_of(hash_product(x), shift);
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
