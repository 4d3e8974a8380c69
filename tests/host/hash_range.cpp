// Host-side check of the count kernel's cuckoo hash functions (tc_hash.h): every
// slot index must lie in [0, 2^b) for every table size the kernel uses, for all
// ids below 2^24 (narrow variant) and a dense sample of 31-bit ids (wide
// variant).  Also reports how evenly the narrow hash spreads consecutive ids,
// and how often cuckoo insertion (the kernel's rule: alternate halves, at most
// 48 kicks) leaves a key for the stash when the ids sit in a window 16 times
// the key count, as the small graphs of a packed batch do.
#include <stdio.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

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
  // stash use for clustered ids: keys distinct, uniform in [base, base + 16 * keys)
  long tables = 0, stashed = 0;
  uint64_t lcg = 12345;
  auto next = [&]() { lcg = lcg * 6364136223846793005ull + 1442695040888963407ull; return (uint32_t)(lcg >> 33); };
  for (int keys : {16, 40, 64, 96}) {
    int b = 4;
    while ((1 << b) < keys + (keys >> 2) + 1) ++b;
    const int side = 1 << b, shift = 32 - b;
    for (int trial = 0; trial < 2000; ++trial) {
      const uint32_t base = next() % (1u << 23);
      std::vector<int32_t> ks;
      while ((int)ks.size() < keys) {
        const int32_t k = (int32_t)(base + next() % (16u * keys));
        if (std::find(ks.begin(), ks.end(), k) == ks.end()) ks.push_back(k);
      }
      std::vector<int32_t> slot(2 * side, -1);
      int left = 0;
      for (int32_t k : ks) {
        int32_t cur = k;
        int hs = 0;
        for (int kick = 0; kick < 48 && cur != -1; ++kick) {
          const uint32_t s = hs ? side + tc::hash_b<false>(cur, shift) : tc::hash_a<false>(cur, shift);
          std::swap(cur, slot[s]);
          hs ^= 1;
        }
        left += cur != -1;
      }
      ++tables;
      stashed += left > 0;
    }
  }
  const double stash_rate = (double)stashed / (double)tables;
  if (stash_rate > 0.05) ++bad;
  printf("stash_rate=%.4f\n", stash_rate);
  printf("out_of_range=%ld max_load=%d\n", bad, mx);
  return bad == 0 ? 0 : 1;
}
