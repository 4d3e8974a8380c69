// tc_device.h - device-side helpers shared by the gfx950 kernels of libtc.
//
// Everything here targets CDNA wave64 directly: ballots are 64-bit, lane ranks
// come from mbcnt, and wave-local LDS hand-offs are ordered with wavefront-scope
// fences (a wave's LDS operations complete in order once lgkmcnt drains).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of `mask` at lanes below the calling lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t popc(uint64_t mask) { return (uint32_t)__popcll(mask); }

// XCD-aware tile order.  Workgroups go to the eight XCDs round robin (workgroup
// b to XCD b mod 8), and each XCD has its own L2.  Giving every XCD one
// contiguous range of tiles, taken in order, means that the cache line where
// one tile's output ends and the next tile's begins is usually written through
// one L2 rather than two.
constexpr int kXcds = 8;

// The tile of workgroup b when a launch has one workgroup per tile (g tiles).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t g) {
  const int64_t per = g / kXcds, rem = g % kXcds;
  const int64_t x = b % kXcds, i = b / kXcds;
  return x * per + (x < rem ? x : rem) + i;
}

// Make this wave's earlier LDS writes visible to its later LDS reads from other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast lane `src`'s value (src wave-uniform) to the whole wave.
__device__ __forceinline__ int32_t read_lane(int32_t v, int src) {
  return __builtin_amdgcn_readlane(v, src);
}
__device__ __forceinline__ int64_t read_lane64(int64_t v, int src) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(uint64_t)v, src);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int32_t first_lane(int32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// Inclusive wave scan (sum) of a 64-bit value.
__device__ __forceinline__ int64_t wave_inclusive_sum(int64_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int64_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

// 32-bit inclusive wave scans on DPP lane moves, which need no LDS round trip
// (a shuffle is a ds_bpermute).  Kogge-Stone inside each row of 16 lanes
// (row_shr 1, 2, 4, 8), then row_bcast:15 carries row 0 into row 1 and row 2
// into row 3, and row_bcast:31 carries lanes 0-31 into rows 2 and 3.  A lane
// whose source lies outside its row, or that the row mask leaves out, gets the
// identity (bound_ctrl off: the destination keeps `old`).  Called by the whole
// wave.
namespace dpp {
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;
}  // namespace dpp

template <typename Op>
__device__ __forceinline__ int32_t wave_inclusive_scan32(int32_t x, int32_t identity, Op op) {
  x = op(x, __builtin_amdgcn_update_dpp(identity, x, dpp::kRowShr1, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(identity, x, dpp::kRowShr2, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(identity, x, dpp::kRowShr4, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(identity, x, dpp::kRowShr8, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(identity, x, dpp::kRowBcast15, 0xa, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(identity, x, dpp::kRowBcast31, 0xc, 0xf, false));
  return x;
}

__device__ __forceinline__ int32_t wave_inclusive_sum32(int32_t x) {
  return wave_inclusive_scan32(x, 0, [](int32_t a, int32_t b) { return a + b; });
}

__device__ __forceinline__ int32_t wave_inclusive_max32(int32_t x) {
  return wave_inclusive_scan32(x, INT32_MIN, [](int32_t a, int32_t b) { return a > b ? a : b; });
}

__device__ __forceinline__ int64_t wave_sum(int64_t x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

template <typename T>
__device__ __forceinline__ T load_off(const void* p, int64_t i);
template <>
__device__ __forceinline__ int32_t load_off<int32_t>(const void* p, int64_t i) {
  return static_cast<const int32_t*>(p)[i];
}
template <>
__device__ __forceinline__ int64_t load_off<int64_t>(const void* p, int64_t i) {
  return static_cast<const int64_t*>(p)[i];
}

}  // namespace tc
