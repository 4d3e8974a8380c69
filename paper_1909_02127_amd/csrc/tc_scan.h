// tc_scan.h - device-wide exclusive scan (reduce-then-scan, three launches).
//
// Values come from a Load functor (int64 result for index i) and prefixes go to
// a Store functor, so callers scan derived quantities (flags, degrees, digit
// counts) without materialising them.  Tiles of kScanTile elements are walked
// as kScanItems coalesced rounds of kScanBlock threads.  The grand total lands
// in partial[num_tiles] for later kernels to read on the device.
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

template <class Op>
__device__ __forceinline__ int64_t wave_inclusive(int64_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int64_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x = Op::apply(y, x);
  }
  return x;
}

// Exclusive scan of one value per thread across the block; *block_total gets the
// combination of all kScanBlock values.  Contains barriers: all threads must call.
template <class Op>
__device__ __forceinline__ int64_t block_exclusive(int64_t x, int64_t* block_total) {
  __shared__ int64_t wave_tot[kScanBlock / kWave];
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  int64_t inc = wave_inclusive<Op>(x);
  if (lane == kWave - 1) wave_tot[wave] = inc;
  __syncthreads();
  int64_t before = Op::identity();
  int64_t all = Op::identity();
#pragma unroll
  for (int w = 0; w < kScanBlock / kWave; ++w) {
    if (w < wave) before = Op::apply(before, wave_tot[w]);
    all = Op::apply(all, wave_tot[w]);
  }
  __syncthreads();
  int64_t exc = __shfl_up(inc, 1, kWave);
  if (lane == 0) exc = Op::identity();
  *block_total = all;
  return Op::apply(before, exc);
}

template <class Op, class Load>
__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(int64_t len, Load load,
                                                                  int64_t* partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t acc = Op::identity();
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + (int64_t)r * kScanBlock + threadIdx.x;
    if (i < len) acc = Op::apply(acc, load(i));
  }
  int64_t total;
  (void)block_exclusive<Op>(acc, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

template <class Op>
__global__ __launch_bounds__(1024) void scan_partials_kernel(int64_t num, int64_t* partial) {
  __shared__ int64_t wave_tot[1024 / kWave];
  __shared__ int64_t carry_s;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) carry_s = Op::identity();
  __syncthreads();
  for (int64_t base = 0; base < num; base += 1024) {
    int64_t i = base + threadIdx.x;
    int64_t x = i < num ? partial[i] : Op::identity();
    int64_t inc = wave_inclusive<Op>(x);
    if (lane == kWave - 1) wave_tot[wave] = inc;
    __syncthreads();
    int64_t before = carry_s, all = carry_s;
    for (int w = 0; w < 1024 / kWave; ++w) {
      if (w < wave) before = Op::apply(before, wave_tot[w]);
      all = Op::apply(all, wave_tot[w]);
    }
    int64_t exc = __shfl_up(inc, 1, kWave);
    if (lane == 0) exc = Op::identity();
    if (i < num) partial[i] = Op::apply(before, exc);
    __syncthreads();
    if (threadIdx.x == 0) carry_s = all;
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[num] = carry_s;
}

template <class Op, class Load, class Store>
__global__ __launch_bounds__(kScanBlock) void scan_down_kernel(int64_t len, Load load, Store store,
                                                                const int64_t* partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t carry = partial[blockIdx.x];
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + (int64_t)r * kScanBlock + threadIdx.x;
    int64_t x = i < len ? load(i) : Op::identity();
    int64_t total;
    int64_t exc = block_exclusive<Op>(x, &total);
    if (i < len) store(i, Op::apply(carry, exc));
    carry = Op::apply(carry, total);
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
