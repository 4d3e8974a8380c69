// tc_scan.h - device-wide exclusive scan (reduce-then-scan, three launches).
//
// Values come from a Load functor (int64 result for index i) and prefixes go to
// a Store functor, so callers scan derived quantities (flags, degrees, digit
// counts) without materialising them.  A tile of kScanTile elements is four
// wave-owned runs of kScanItems coalesced 64-wide rounds.  The grand total
// lands in partial[num_tiles] for later kernels to read on the device.
#pragma once

#include "tc_device.h"

namespace tc {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;

struct OpSum {
  static __device__ __forceinline__ int64_t identity() { return 0; }
  static __device__ __forceinline__ int64_t apply(int64_t a, int64_t b) { return a + b; }
};
struct OpMin {
  static __device__ __forceinline__ int64_t identity() { return INT64_MAX; }
  static __device__ __forceinline__ int64_t apply(int64_t a, int64_t b) { return a < b ? a : b; }
};

inline int64_t scan_num_tiles(int64_t len) { return (len + kScanTile - 1) / kScanTile; }
// int64 entries the caller must provide as `partial` for a scan of `len` values.
inline int64_t scan_partial_len(int64_t len) { return scan_num_tiles(len) + 1; }

// A 64-bit DPP lane move (two 32-bit moves): lanes without a source under
// control Ctrl, or outside RowMask, get `old` (bound_ctrl off).
template <int Ctrl, int RowMask>
__device__ __forceinline__ int64_t dpp_move64(int64_t old, int64_t x) {
  const uint64_t o = (uint64_t)old, v = (uint64_t)x;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)v,
                                                            Ctrl, RowMask, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
      (int)(uint32_t)(o >> 32), (int)(uint32_t)(v >> 32), Ctrl, RowMask, 0xf, false);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Inclusive wave scan on DPP moves (no LDS round trips): Kogge-Stone inside
// each row of 16 lanes, then row_bcast:15 and row_bcast:31 carry the row
// prefixes across rows.  Called by the whole wave.
template <class Op>
__device__ __forceinline__ int64_t wave_inclusive(int64_t x) {
  const int64_t id = Op::identity();
  x = Op::apply(dpp_move64<dpp::kRowShr1, 0xf>(id, x), x);
  x = Op::apply(dpp_move64<dpp::kRowShr2, 0xf>(id, x), x);
  x = Op::apply(dpp_move64<dpp::kRowShr4, 0xf>(id, x), x);
  x = Op::apply(dpp_move64<dpp::kRowShr8, 0xf>(id, x), x);
  x = Op::apply(dpp_move64<dpp::kRowBcast15, 0xa>(id, x), x);
  x = Op::apply(dpp_move64<dpp::kRowBcast31, 0xc>(id, x), x);
  return x;
}

// The value of lane l - 1 (lane 0: the identity), by a whole-wave DPP shift
// (wave_shr:1).  Called by the whole wave.
template <class Op>
__device__ __forceinline__ int64_t wave_exclusive_from_inclusive(int64_t inc) {
  constexpr int kWaveShr1 = 0x138;
  return dpp_move64<kWaveShr1, 0xf>(Op::identity(), inc);
}

// Combination of one value per lane across the wave (every lane gets it).
template <class Op>
__device__ __forceinline__ int64_t wave_reduce(int64_t x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x = Op::apply(x, __shfl_xor(x, off, kWave));
  return x;
}

// Each wave of a tile owns kScanItems consecutive rounds of 64 elements, so a
// tile needs one workgroup barrier (to combine the four wave totals).
template <class Op, class Load>
__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(int64_t len, Load load,
                                                                  int64_t* partial) {
  __shared__ int64_t wave_tot[kScanBlock / kWave];
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)wave * kScanItems * kWave;
  int64_t acc = Op::identity();
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)r * kWave + lane;
    if (i < len) acc = Op::apply(acc, load(i));
  }
  acc = wave_reduce<Op>(acc);
  if (lane == 0) wave_tot[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t total = Op::identity();
    for (int w = 0; w < kScanBlock / kWave; ++w) total = Op::apply(total, wave_tot[w]);
    partial[blockIdx.x] = total;
  }
}

// The tile totals, scanned in place by one workgroup: each round covers 1024
// threads x kPartialItems consecutive totals (a serial scan per thread, then
// one scan of the thread sums).  partial[num] receives the grand total.
constexpr int kPartialItems = 8;

template <class Op>
__global__ __launch_bounds__(1024) void scan_partials_kernel(int64_t num, int64_t* partial) {
  __shared__ int64_t wave_tot[1024 / kWave];
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  int64_t carry = Op::identity();
  for (int64_t base = 0; base < num; base += 1024 * kPartialItems) {
    const int64_t first = base + (int64_t)threadIdx.x * kPartialItems;
    int64_t x[kPartialItems];
    int64_t mine = Op::identity();
#pragma unroll
    for (int k = 0; k < kPartialItems; ++k) {
      x[k] = first + k < num ? partial[first + k] : Op::identity();
      mine = Op::apply(mine, x[k]);
    }
    const int64_t inc = wave_inclusive<Op>(mine);
    if (lane == kWave - 1) wave_tot[wave] = inc;
    __syncthreads();
    int64_t before = carry, all = carry;
    for (int w = 0; w < 1024 / kWave; ++w) {
      if (w < wave) before = Op::apply(before, wave_tot[w]);
      all = Op::apply(all, wave_tot[w]);
    }
    const int64_t exc = wave_exclusive_from_inclusive<Op>(inc);
    int64_t run = Op::apply(before, exc);
#pragma unroll
    for (int k = 0; k < kPartialItems; ++k) {
      if (first + k < num) partial[first + k] = run;
      run = Op::apply(run, x[k]);
    }
    carry = all;
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[num] = carry;
}

template <class Op, class Load, class Store>
__global__ __launch_bounds__(kScanBlock) void scan_down_kernel(int64_t len, Load load, Store store,
                                                                const int64_t* partial) {
  __shared__ int64_t wave_tot[kScanBlock / kWave];
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)wave * kScanItems * kWave;
  int64_t x[kScanItems];
  int64_t acc = Op::identity();
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)r * kWave + lane;
    x[r] = i < len ? load(i) : Op::identity();
    acc = Op::apply(acc, x[r]);
  }
  acc = wave_reduce<Op>(acc);
  if (lane == 0) wave_tot[wave] = acc;
  __syncthreads();
  int64_t carry = partial[blockIdx.x];
  for (int w = 0; w < wave; ++w) carry = Op::apply(carry, wave_tot[w]);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)r * kWave + lane;
    const int64_t inc = wave_inclusive<Op>(x[r]);
    const int64_t exc = wave_exclusive_from_inclusive<Op>(inc);
    if (i < len) store(i, Op::apply(carry, exc));
    carry = Op::apply(carry, read_lane64(inc, kWave - 1));
  }
}

// Enqueue the scan on `stream`.  partial: device int64[scan_partial_len(len)].
template <class Op, class Load, class Store>
hipError_t scan_exclusive(int64_t len, Load load, Store store, int64_t* partial,
                          hipStream_t stream) {
  const int64_t tiles = scan_num_tiles(len);
  if (tiles > 0) {
    scan_reduce_kernel<Op, Load><<<dim3((unsigned)tiles), dim3(kScanBlock), 0, stream>>>(
        len, load, partial);
  }
  scan_partials_kernel<Op><<<1, 1024, 0, stream>>>(tiles, partial);
  if (tiles > 0) {
    scan_down_kernel<Op, Load, Store><<<dim3((unsigned)tiles), dim3(kScanBlock), 0, stream>>>(
        len, load, store, partial);
  }
  return hipGetLastError();
}

}  // namespace tc
