// Host-side check of the count kernel's cuckoo hash functions (tc_hash.h): every
// slot index must lie in [0, 2^b) for every table size the kernel uses, for all
// ids below 2^24 (narrow variant) and a dense sample of 31-bit ids (wide
// variant).  Also reports how evenly the narrow hash spreads consecutive ids.
#include <stdio.h>
#include <stdint.h>

#include "tc_hash.h"

int main() {
  long bad = 0;
  for (int b = 4; b <= 11; ++b) {
    const int shift = 32 - b;
    const uint32_t side = 1u << b;
    for (int32_t k = 0; k < (1 << 24); ++k) {
      if (tc::hash_a<false>(k, shift) >= side || tc::hash_b<false>(k, shift) >= side) ++bad;
    }
    for (int64_t k = 0; k < ((int64_t)1 << 31); k += 4099) {
      if (tc::hash_a<true>((int32_t)k, shift) >= side || tc::hash_b<true>((int32_t)k, shift) >= side)
        ++bad;
    }
    // the smallest id whose 24-bit product with kHashA24 has bit 31 set; a
    // signed shift of that product gives a negative slot
    if (tc::hash_a<false>(208, shift) >= side) ++bad;
  }
  // the wide variant spreads a block of consecutive ids above 2^24 as well
  {
    int wload[1024] = {0}, wmx = 0;
    for (int32_t k = (1 << 25) + 12345; k < (1 << 25) + 12345 + 1024; ++k) {
      int s = (int)tc::hash_a<true>(k, 22);
      if (++wload[s] > wmx) wmx = wload[s];
    }
    if (wmx > 8) ++bad;
  }
  // balance: 1024 consecutive ids into 1024 slots, max load per slot
  int load[1024] = {0}, mx = 0;
  for (int32_t k = 0; k < 1024; ++k) {
    int s = (int)tc::hash_a<false>(k, 22);
    if (++load[s] > mx) mx = load[s];
  }
  printf("out_of_range=%ld max_load=%d\n", bad, mx);
  return bad == 0 ? 0 : 1;
}
