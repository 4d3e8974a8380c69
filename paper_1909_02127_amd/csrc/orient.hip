// orient.hip - tc_orient: keep each undirected edge once, from lower to higher rank.
//
// This is the unique mapping order of Alg. 1 ("Generate_UMO") and Sec. III-A:
// the triangle query is a single neighbourhood-equivalence class, so its nodes
// are visited in increasing order and every triangle is matched once.  Any
// strict total order works; the default ranks by (degree, id), which keeps every
// out-degree O(sqrt(m)) so N+(u) fits in LDS during counting.  TC_ORDER_ID is
// the paper's own "destination id larger than source id" rule.
//
// Orientation is a stream compaction of the symmetric column array: rows are
// stored in order and each row's entries in order, so the DAG position of a kept
// entry is the number of kept entries before it in the whole array, and
// dag_row_ptr[u] is that count at row_ptr[u].  The entries are cut into tiles of
// kTile consecutive positions, whatever the row boundaries, so a hub row is
// spread over many workgroups and a tile of short rows costs the same as a tile
// of one long row:
//   rows   deg[u], and for every tile the first row starting at or after it
//   flags  per tile: the row of each entry (segment-start markers + max-scan),
//          the keep bit of each entry, the kept count
//   scan   exclusive scan of the tile counts
//   write  per tile: the kept entries compacted through LDS and written
//          contiguously, and dag_row_ptr of the rows starting in the tile
#include "tc_device.h"
#include "tc_host.h"
#include "tc_scan.h"

#include <algorithm>

namespace tc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kItems = 16;              // entries per thread and tile
constexpr int kTile = kBlock * kItems;  // entries per tile
constexpr int kPadded = kTile + kTile / kItems;
constexpr int kTileBlocksPerCu = 64;    // write_kernel grid cap (LDS: about 35 KB per workgroup)
constexpr int kFlagBlocksPerCu = 64;    // flags_kernel grid cap: one tile per workgroup up to 64 per CU

// LDS index of tile entry i, padded so that a thread's kItems consecutive
// entries fall into distinct banks across a wave.
__device__ __forceinline__ int padded(int i) { return i + i / kItems; }
static_assert(kItems <= 16, "keep bits are stored 16 per thread");

struct TileInfo {
  int64_t nnz;        // row_ptr[n]
  int64_t num_tiles;  // ceil(nnz / kTile)
  int32_t over;       // nnz needs more tiles than the workspace provides
  int32_t pad[3];
};

template <typename OffT, int Order>
__global__ __launch_bounds__(256) void rows_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                   int32_t* __restrict__ deg,
                                                   int32_t* __restrict__ row_start,
                                                   int64_t tiles_max, TileInfo* __restrict__ info) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += stride) {
    const int64_t here = row_ptr[u];
    if (Order == TC_ORDER_DEGREE && u < n) deg[u] = (int32_t)(row_ptr[u + 1] - here);
    // the tiles t with row_ptr[u-1] < t * kTile <= row_ptr[u] first reach row u
    const int64_t t0 = u == 0 ? 0 : (int64_t)row_ptr[u - 1] / kTile + 1;
    int64_t t1 = here / kTile;
    if (t1 > tiles_max) t1 = tiles_max;
    for (int64_t t = t0; t <= t1; ++t) row_start[t] = (int32_t)u;
    if (u == n) {
      const int64_t tiles = (here + kTile - 1) / kTile;
      info->nnz = here;
      info->num_tiles = tiles;
      info->over = tiles > tiles_max;
    }
  }
}

// Block-wide exclusive max-scan of one int32 per thread (-1 before the first).
// Contains barriers: all threads call.
__device__ __forceinline__ int32_t block_exclusive_max(int32_t x, int32_t* wave_tot) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int32_t inc = wave_inclusive_max32(x);
  if (lane == kWave - 1) wave_tot[wave] = inc;
  __syncthreads();
  int32_t before = -1;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w)
    if (w < wave) before = before > wave_tot[w] ? before : wave_tot[w];
  __syncthreads();
  int32_t exc = __shfl_up(inc, 1, kWave);
  if (lane == 0) exc = -1;
  return before > exc ? before : exc;
}

// Block-wide exclusive sum of one int32 per thread; *total gets the sum.
// Contains barriers: all threads call.
__device__ __forceinline__ int32_t block_exclusive_sum(int32_t x, int32_t* wave_tot,
                                                       int32_t* total) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int32_t inc = wave_inclusive_sum32(x);
  if (lane == kWave - 1) wave_tot[wave] = inc;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    if (w < wave) before += wave_tot[w];
    all += wave_tot[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

// The tile's entries into LDS with coalesced reads (entry i at padded(i)).  The
// reads are clamped to the tile's last entry (len >= 1) rather than guarded, so
// all of them are in flight at once.
__device__ __forceinline__ void load_tile(const int32_t* __restrict__ col, int64_t e0, int len,
                                          int32_t* sval) {
  int32_t v[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int i = k * kBlock + (int)threadIdx.x;
    v[k] = col[e0 + (i < len ? i : len - 1)];
  }
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int i = k * kBlock + (int)threadIdx.x;
    sval[padded(i)] = i < len ? v[k] : 0;
  }
}

// Pass 1: the keep bit of every entry (kItems bits per thread, in entry order)
// and the kept count of every tile.  The entries and their degrees are loaded
// in the coalesced layout (entry k * kBlock + tid in thread tid), all loads in
// flight together; the row of every entry comes from a max-scan over the row
// start markers in the blocked layout (entries tid * kItems + k), and the keep
// test runs back in the coalesced layout with the entry's values at hand.
template <typename OffT, int Order>
__global__ __launch_bounds__(kBlock) void flags_kernel(
    int64_t n, const OffT* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ deg, const int32_t* __restrict__ row_start,
    const TileInfo* __restrict__ info, uint16_t* __restrict__ bits, int32_t* __restrict__ tile_cnt) {
  __shared__ int32_t srow[kPadded];            // row start markers, then the row of every entry
  __shared__ uint32_t skeep[kTile / 4];        // keep flag of every entry, one byte each
  __shared__ int32_t wave_tot[kWavesPerBlock];
  if (info->over) return;
  const int64_t num_tiles = info->num_tiles, nnz = info->nnz;
  const int tid = threadIdx.x;
  uint8_t* keep8 = reinterpret_cast<uint8_t*>(skeep);
  for (int64_t t = blockIdx.x; t < num_tiles; t += gridDim.x) {
    const int64_t e0 = t * kTile;
    const int len = (int)(nnz - e0 < kTile ? nnz - e0 : kTile);  // >= 1
    const int32_t r_lo = row_start[t];
    const int64_t r_hi = t + 1 < num_tiles ? (int64_t)row_start[t + 1] : n;
    int32_t v[kItems], dv[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int i = k * kBlock + tid;
      v[k] = col[e0 + (i < len ? i : len - 1)];
    }
    if (Order == TC_ORDER_DEGREE) {
#pragma unroll
      for (int k = 0; k < kItems; ++k) dv[k] = deg[v[k]];
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) srow[padded(k * kBlock + tid)] = -1;
    __syncthreads();
    // each non-empty row starting in the tile marks its first entry
    for (int64_t u = r_lo + tid; u < r_hi; u += kBlock) {
      const int64_t b = (int64_t)row_ptr[u] - e0;
      if (row_ptr[u + 1] > row_ptr[u] && b >= 0 && b < len) srow[padded((int)b)] = (int32_t)u;
    }
    __syncthreads();
    {
      int32_t mk[kItems];
      int32_t agg = -1;
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        mk[k] = srow[padded(tid * kItems + k)];
        agg = agg > mk[k] ? agg : mk[k];
      }
      // entries before the tile's first marker belong to the row before r_lo
      int32_t cur = block_exclusive_max(agg, wave_tot);
      cur = cur > r_lo - 1 ? cur : r_lo - 1;
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        cur = cur > mk[k] ? cur : mk[k];
        srow[padded(tid * kItems + k)] = cur;
      }
    }
    __syncthreads();
    {
      // rank(u) < rank(v); the row degrees are all loaded before any is used,
      // and the test has no short-circuit branches
      int32_t u[kItems], du[kItems];
#pragma unroll
      for (int k = 0; k < kItems; ++k) u[k] = srow[padded(k * kBlock + tid)];
      if (Order == TC_ORDER_DEGREE) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) du[k] = deg[u[k] > 0 ? u[k] : 0];
      }
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const int i = k * kBlock + tid;
        bool keep = u[k] < v[k];
        if (Order == TC_ORDER_DEGREE) keep = (du[k] < dv[k]) | ((du[k] == dv[k]) & keep);
        keep8[i] = (uint8_t)((i < len) & (u[k] >= 0) & keep);
      }
    }
    __syncthreads();
    // the thread's kItems consecutive flags as bits
    uint32_t mask = 0;
#pragma unroll
    for (int q = 0; q < kItems / 4; ++q) {
      const uint32_t w = skeep[tid * (kItems / 4) + q];
#pragma unroll
      for (int j = 0; j < 4; ++j) mask |= ((w >> (8 * j)) & 1u) << (4 * q + j);
    }
    bits[t * kBlock + tid] = (uint16_t)mask;
    int32_t kept;
    (void)block_exclusive_sum((int32_t)popc(mask), wave_tot, &kept);
    if (tid == 0) tile_cnt[t] = kept;
    __syncthreads();
  }
}

struct TileCountLoad {
  const int32_t* cnt;
  const TileInfo* info;
  __device__ int64_t operator()(int64_t i) const {
    return (!info->over && i < info->num_tiles) ? cnt[i] : 0;
  }
};
struct TileOffStore {
  int64_t* off;
  __device__ void operator()(int64_t i, int64_t p) const { off[i] = p; }
};

__global__ void finalize_kernel(const int64_t* total, const TileInfo* info, int64_t cap,
                                int64_t* m_out) {
  const int64_t m = *total;
  *m_out = (info->over || m > cap) ? -(int64_t)TC_ERR_CAPACITY : m;
}

// Pass 2: compact each tile's kept entries through LDS, write them contiguously
// at the tile's offset, and write dag_row_ptr of the rows starting in the tile
// (the last tile also takes the rows starting at nnz, through index n).
template <typename OffT>
__global__ __launch_bounds__(kBlock) void write_kernel(
    int64_t n, const OffT* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ row_start, const TileInfo* __restrict__ info,
    const uint16_t* __restrict__ bits, const int64_t* __restrict__ tile_off,
    const int64_t* __restrict__ m_out, OffT* __restrict__ dag_ptr, int32_t* __restrict__ dag_col) {
  __shared__ int32_t sval[kPadded];
  __shared__ int32_t stage[kTile];
  __shared__ int32_t toff[kBlock];
  __shared__ uint32_t tmask[kBlock];
  __shared__ int32_t wave_tot[kWavesPerBlock];
  if (*m_out < 0) return;
  const int64_t num_tiles = info->num_tiles, nnz = info->nnz;
  const int tid = threadIdx.x;
  if (num_tiles == 0) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t u = (int64_t)blockIdx.x * kBlock + tid; u <= n; u += stride) dag_ptr[u] = 0;
    return;
  }
  for (int64_t t = blockIdx.x; t < num_tiles; t += gridDim.x) {
    const int64_t e0 = t * kTile;
    const int len = (int)(nnz - e0 < kTile ? nnz - e0 : kTile);
    const int32_t r_lo = row_start[t];
    const int64_t r_hi = t + 1 < num_tiles ? (int64_t)row_start[t + 1] : n + 1;
    const int64_t base = tile_off[t];
    const uint32_t mask = bits[t * kBlock + tid];
    load_tile(col, e0, len, sval);
    int32_t kept;
    const int32_t before = block_exclusive_sum((int32_t)popc(mask), wave_tot, &kept);
    toff[tid] = before;
    tmask[tid] = mask;
    int32_t p = before;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
      if ((mask >> k) & 1u) stage[p++] = sval[padded(tid * kItems + k)];
    __syncthreads();
    for (int j = tid; j < kept; j += kBlock) dag_col[base + j] = stage[j];
    for (int64_t u = r_lo + tid; u < r_hi; u += kBlock) {
      const int64_t pos = (int64_t)row_ptr[u] - e0;  // in [0, len]
      int32_t kb = kept;
      if (pos >= 0 && pos < len) {
        const int q = (int)pos / kItems;
        kb = toff[q] + (int32_t)__popc(tmask[q] & ((1u << ((int)pos % kItems)) - 1u));
      }
      dag_ptr[u] = (OffT)(base + kb);
    }
    __syncthreads();
  }
}

template <typename OffT>
__global__ void zero_on_error_kernel(OffT* p, int64_t len, const int64_t* m_out) {
  if (*m_out >= 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0;
}

// Tiles the workspace provides for: a symmetric CSR whose DAG fits `cap` edges
// has nnz <= 2 cap, and a simple graph has nnz <= n (n - 1).
int64_t tiles_for(int64_t n, int64_t cap) {
  const int64_t by_cap = (2 * cap + kTile - 1) / kTile;
  const int64_t by_n = (n * (n - 1) + kTile - 1) / kTile;  // n < 2^31: no overflow
  return std::min(by_cap, by_n);
}

struct OrientLayout {
  int32_t* deg;
  int32_t* row_start;
  TileInfo* info;
  uint16_t* bits;
  int32_t* tile_cnt;
  int64_t* tile_off;
  int64_t* partial;
  int64_t tiles_max;
  size_t bytes;
};

OrientLayout carve_orient(void* ws, int64_t n, int64_t cap) {
  Carver c(ws);
  OrientLayout L;
  L.tiles_max = tiles_for(n, cap);
  L.deg = c.take<int32_t>(n);
  L.row_start = c.take<int32_t>(L.tiles_max + 1);
  L.info = c.take<TileInfo>(1);
  L.bits = c.take<uint16_t>(L.tiles_max * kBlock);
  L.tile_cnt = c.take<int32_t>(L.tiles_max);
  L.tile_off = c.take<int64_t>(L.tiles_max);
  L.partial = c.take<int64_t>(scan_partial_len(L.tiles_max));
  L.bytes = c.used();
  return L;
}

template <typename OffT, int Order>
tc_status orient_impl(int64_t n, const OffT* row_ptr, const int32_t* col, OffT* dag_ptr,
                      int32_t* dag_col, int64_t cap, int64_t* m_out, const OrientLayout& L,
                      hipStream_t s) {
  const int grid_tiles = (int)std::max<int64_t>(
      1, std::min<int64_t>(L.tiles_max, (int64_t)kTileBlocksPerCu * device_cu_count()));
  rows_kernel<OffT, Order><<<grid_for(n + 1, 256, 8192), 256, 0, s>>>(n, row_ptr, L.deg,
                                                                       L.row_start, L.tiles_max,
                                                                       L.info);
  const int grid_flags = (int)std::max<int64_t>(
      1, std::min<int64_t>(L.tiles_max, (int64_t)kFlagBlocksPerCu * device_cu_count()));
  flags_kernel<OffT, Order><<<grid_flags, kBlock, 0, s>>>(n, row_ptr, col, L.deg, L.row_start,
                                                          L.info, L.bits, L.tile_cnt);
  hipError_t e = scan_exclusive<OpSum>(L.tiles_max, TileCountLoad{L.tile_cnt, L.info},
                                       TileOffStore{L.tile_off}, L.partial, s);
  if (e != hipSuccess) return check_hip(e, "orient tile scan");
  finalize_kernel<<<1, 1, 0, s>>>(L.partial + scan_num_tiles(L.tiles_max), L.info, cap, m_out);
  write_kernel<OffT><<<grid_tiles, kBlock, 0, s>>>(n, row_ptr, col, L.row_start, L.info, L.bits,
                                                   L.tile_off, m_out, dag_ptr, dag_col);
  zero_on_error_kernel<OffT><<<grid_for(n + 1, 256, 4096), 256, 0, s>>>(dag_ptr, n + 1, m_out);
  return check_hip(hipGetLastError(), "tc_orient launch");
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_orient(const tc_csr* sym, int32_t order, void* dag_row_ptr,
                               int32_t* dag_col, int64_t dag_col_capacity, int64_t* m_out,
                               void* ws, size_t* ws_bytes, void* stream) {
  using namespace tc;
  if (!sym) return fail(TC_ERR_INVALID_ARG, "sym is NULL");
  const int64_t n = sym->n;
  if (n < 0 || dag_col_capacity < 0) return fail(TC_ERR_INVALID_ARG, "negative size");
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (dag_col_capacity > ((int64_t)1 << 40))
    return fail(TC_ERR_UNSUPPORTED, "dag_col_capacity=%lld is beyond 2^40",
                (long long)dag_col_capacity);
  if (sym->offset_bytes != 4 && sym->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", sym->offset_bytes);
  if (order != TC_ORDER_DEGREE && order != TC_ORDER_ID)
    return fail(TC_ERR_INVALID_ARG, "unknown order %d", order);
  tc_status st;
  if (workspace_query(ws, ws_bytes, carve_orient(nullptr, n, dag_col_capacity).bytes, &st))
    return st;
  if (!sym->row_ptr || !dag_row_ptr || !m_out || (dag_col_capacity > 0 && !dag_col))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const OrientLayout L = carve_orient(ws, n, dag_col_capacity);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (sym->offset_bytes == 4) {
    auto rp = static_cast<const int32_t*>(sym->row_ptr);
    auto dp = static_cast<int32_t*>(dag_row_ptr);
    st = order == TC_ORDER_DEGREE
             ? orient_impl<int32_t, TC_ORDER_DEGREE>(n, rp, sym->col, dp, dag_col,
                                                     dag_col_capacity, m_out, L, s)
             : orient_impl<int32_t, TC_ORDER_ID>(n, rp, sym->col, dp, dag_col, dag_col_capacity,
                                                 m_out, L, s);
  } else {
    auto rp = static_cast<const int64_t*>(sym->row_ptr);
    auto dp = static_cast<int64_t*>(dag_row_ptr);
    st = order == TC_ORDER_DEGREE
             ? orient_impl<int64_t, TC_ORDER_DEGREE>(n, rp, sym->col, dp, dag_col,
                                                     dag_col_capacity, m_out, L, s)
             : orient_impl<int64_t, TC_ORDER_ID>(n, rp, sym->col, dp, dag_col, dag_col_capacity,
                                                 m_out, L, s);
  }
  return st == TC_OK ? ok() : st;
}
