// orient.hip - tc_orient: keep each undirected edge once, from lower to higher rank.
//
// This is the unique mapping order of Alg. 1 ("Generate_UMO") and Sec. III-A:
// the triangle query is a single neighbourhood-equivalence class, so its nodes
// are visited in increasing order and every triangle is matched once.  Any
// strict total order works; the default ranks by (degree, id), which keeps every
// out-degree O(sqrt(m)) so N+(u) fits in LDS during counting.  TC_ORDER_ID is
// the paper's own "destination id larger than source id" rule.
//
// Pass 1 counts kept entries per row, a scan turns the counts into the DAG's
// row offsets, pass 2 writes the kept entries in row order (ballot + mbcnt keeps
// the order).  A wave takes four rows at a time: when all four have at most
// kShortRow entries it gives each 16 lanes, otherwise it walks them one after
// the other with all 64 lanes.  Rows longer than kLongRow are queued and walked
// by a whole workgroup.
#include "tc_device.h"
#include "tc_host.h"
#include "tc_scan.h"

#include <algorithm>

namespace tc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int64_t kLongRow = 2048;
constexpr int32_t kShortRow = 64;
constexpr int kGroup = 16;  // lanes per short row
constexpr int kGroupsPerWave = kWave / kGroup;

template <typename OffT>
__global__ __launch_bounds__(256) void degree_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                     int32_t* __restrict__ deg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    deg[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
}

template <int Order>
__device__ __forceinline__ bool keep_edge(int64_t u, int32_t du, int32_t v,
                                          const int32_t* __restrict__ deg) {
  if (Order == TC_ORDER_ID) return u < v;
  const int32_t dv = deg[v];
  return du < dv || (du == dv && u < v);
}

// Largest length among the four 16-lane groups of a wave (uniform).
__device__ __forceinline__ int32_t group_max(int32_t len) {
  int32_t a = read_lane(len, 0), b = read_lane(len, 16), c = read_lane(len, 32),
          d = read_lane(len, 48);
  a = a > b ? a : b;
  c = c > d ? c : d;
  return a > c ? a : c;
}

__global__ void clear_counter_kernel(int32_t* c) { *c = 0; }

// Pass 1 (rows up to kLongRow): four rows per wave; short rows counted 16 lanes
// each, otherwise one row at a time with the whole wave; long rows are queued.
template <typename OffT, int Order>
__global__ __launch_bounds__(kBlock) void count_rows_kernel(
    int64_t n, const OffT* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ deg, int64_t* __restrict__ outdeg, int32_t* __restrict__ long_rows,
    int32_t* __restrict__ long_count) {
  const int lane = lane_id();
  const int g = lane / kGroup, gl = lane % kGroup;
  const uint64_t gmask = 0xFFFFull << (kGroup * g);
  const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t r0 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * kGroupsPerWave;
       r0 < n; r0 += waves * kGroupsPerWave) {
    const int64_t u = r0 + g;
    int64_t beg = 0, end = 0;
    if (u < n) {
      beg = row_ptr[u];
      end = row_ptr[u + 1];
    }
    const int64_t len64 = end - beg;
    const int32_t len = len64 > kShortRow ? kShortRow + 1 : (int32_t)len64;
    const int32_t widest = group_max(len);
    if (widest <= kShortRow) {
      const int32_t iters = (widest + kGroup - 1) / kGroup;
      uint32_t kept = 0;
      for (int32_t k = 0; k < iters; ++k) {
        const int32_t j = k * kGroup + gl;
        const bool kk = j < len && keep_edge<Order>(u, len, col[beg + j], deg);
        kept += popc(ballot(kk) & gmask);
      }
      if (gl == 0 && u < n) outdeg[u] = kept;
      continue;
    }
    for (int r = 0; r < kGroupsPerWave && r0 + r < n; ++r) {
      const int64_t ur = r0 + r;
      const int64_t rb = read_lane64(beg, r * kGroup), re = read_lane64(end, r * kGroup);
      if (re - rb > kLongRow) {
        if (lane == 0) long_rows[atomicAdd(long_count, 1)] = (int32_t)ur;
        continue;
      }
      const int32_t du = (int32_t)(re - rb);
      uint32_t kept = 0;
      for (int64_t e = rb + lane; e - lane < re; e += kWave) {
        const bool kk = e < re && keep_edge<Order>(ur, du, col[e], deg);
        kept += popc(ballot(kk));
      }
      if (lane == 0) outdeg[ur] = kept;
    }
  }
}

// Pass 1 (long rows): one workgroup per queued row.
template <typename OffT, int Order>
__global__ __launch_bounds__(kBlock) void count_long_kernel(const OffT* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            const int32_t* __restrict__ deg,
                                                            int64_t* __restrict__ outdeg,
                                                            const int32_t* __restrict__ long_rows,
                                                            const int32_t* __restrict__ long_count) {
  __shared__ uint32_t wave_kept[kWavesPerBlock];
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int32_t count = *long_count;
  for (int32_t li = blockIdx.x; li < count; li += gridDim.x) {
    const int64_t u = long_rows[li];
    const int64_t beg = row_ptr[u], end = row_ptr[u + 1];
    const int32_t du = (int32_t)(end - beg);
    uint32_t kept = 0;
    for (int64_t e = beg + threadIdx.x; e - threadIdx.x < end; e += kBlock) {
      const bool k = e < end && keep_edge<Order>(u, du, col[e], deg);
      kept += popc(ballot(k));
    }
    if (lane == 0) wave_kept[wave] = kept;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t s = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) s += wave_kept[w];
      outdeg[u] = s;
    }
    __syncthreads();
  }
}

struct DegLoad {
  const int64_t* outdeg;
  int64_t n;
  __device__ int64_t operator()(int64_t i) const { return i < n ? outdeg[i] : 0; }
};
template <typename OffT>
struct OffStore {
  OffT* dag_ptr;
  __device__ void operator()(int64_t i, int64_t p) const { dag_ptr[i] = (OffT)p; }
};

__global__ void finalize_kernel(const int64_t* total, int64_t cap, int64_t* m_out) {
  const int64_t m = *total;
  *m_out = m > cap ? -(int64_t)TC_ERR_CAPACITY : m;
}

// Pass 2 (rows up to kLongRow): the same walk as pass 1, writing kept entries in
// row order.
template <typename OffT, int Order>
__global__ __launch_bounds__(kBlock) void fill_rows_kernel(
    int64_t n, const OffT* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ deg, const OffT* __restrict__ dag_ptr,
    int32_t* __restrict__ dag_col, const int64_t* __restrict__ m_out) {
  if (*m_out < 0) return;
  const int lane = lane_id();
  const int g = lane / kGroup, gl = lane % kGroup;
  const uint64_t gmask = 0xFFFFull << (kGroup * g);
  const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t r0 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * kGroupsPerWave;
       r0 < n; r0 += waves * kGroupsPerWave) {
    const int64_t u = r0 + g;
    int64_t beg = 0, end = 0, out = 0;
    if (u < n) {
      beg = row_ptr[u];
      end = row_ptr[u + 1];
      out = dag_ptr[u];
    }
    const int64_t len64 = end - beg;
    const int32_t len = len64 > kShortRow ? kShortRow + 1 : (int32_t)len64;
    const int32_t widest = group_max(len);
    if (widest <= kShortRow) {
      const int32_t iters = (widest + kGroup - 1) / kGroup;
      for (int32_t k = 0; k < iters; ++k) {
        const int32_t j = k * kGroup + gl;
        const int32_t v = j < len ? col[beg + j] : 0;
        const bool kk = j < len && keep_edge<Order>(u, len, v, deg);
        const uint64_t m = ballot(kk) & gmask;
        if (kk) dag_col[out + rank_below(m)] = v;
        out += popc(m);
      }
      continue;
    }
    for (int r = 0; r < kGroupsPerWave && r0 + r < n; ++r) {
      const int64_t ur = r0 + r;
      const int64_t rb = read_lane64(beg, r * kGroup), re = read_lane64(end, r * kGroup);
      if (re - rb > kLongRow) continue;
      const int32_t du = (int32_t)(re - rb);
      int64_t o = read_lane64(out, r * kGroup);
      for (int64_t e = rb + lane; e - lane < re; e += kWave) {
        const int32_t v = e < re ? col[e] : 0;
        const bool kk = e < re && keep_edge<Order>(ur, du, v, deg);
        const uint64_t m = ballot(kk);
        if (kk) dag_col[o + rank_below(m)] = v;
        o += popc(m);
      }
    }
  }
}

// Pass 2 (long rows): ordered compaction across the workgroup's four waves.
template <typename OffT, int Order>
__global__ __launch_bounds__(kBlock) void fill_long_kernel(const OffT* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ col,
                                                           const int32_t* __restrict__ deg,
                                                           const OffT* __restrict__ dag_ptr,
                                                           int32_t* __restrict__ dag_col,
                                                           const int32_t* __restrict__ long_rows,
                                                           const int32_t* __restrict__ long_count,
                                                           const int64_t* __restrict__ m_out) {
  if (*m_out < 0) return;
  __shared__ uint32_t wave_kept[kWavesPerBlock];
  const int wave = threadIdx.x / kWave;
  const int32_t count = *long_count;
  for (int32_t li = blockIdx.x; li < count; li += gridDim.x) {
    const int64_t u = long_rows[li];
    const int64_t beg = row_ptr[u], end = row_ptr[u + 1];
    const int32_t du = (int32_t)(end - beg);
    int64_t out = dag_ptr[u];
    for (int64_t e0 = beg; e0 < end; e0 += kBlock) {
      const int64_t e = e0 + threadIdx.x;
      const int32_t v = e < end ? col[e] : 0;
      const bool k = e < end && keep_edge<Order>(u, du, v, deg);
      const uint64_t m = ballot(k);
      if (lane_id() == 0) wave_kept[wave] = popc(m);
      __syncthreads();
      uint32_t before = 0, all = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) {
        if (w < wave) before += wave_kept[w];
        all += wave_kept[w];
      }
      if (k) dag_col[out + before + rank_below(m)] = v;
      out += all;
      __syncthreads();
    }
  }
}

template <typename OffT>
__global__ void zero_on_error_kernel(OffT* p, int64_t len, const int64_t* m_out) {
  if (*m_out >= 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0;
}

struct OrientLayout {
  int32_t* deg;
  int64_t* outdeg;
  int32_t* long_rows;
  int32_t* long_count;
  int64_t* partial;
  size_t bytes;
};

OrientLayout carve_orient(void* ws, int64_t n) {
  Carver c(ws);
  OrientLayout L;
  L.deg = c.take<int32_t>(n);
  L.outdeg = c.take<int64_t>(n);
  L.long_rows = c.take<int32_t>(n);
  L.long_count = c.take<int32_t>(1);
  L.partial = c.take<int64_t>(scan_partial_len(n + 1));
  L.bytes = c.used();
  return L;
}

template <typename OffT, int Order>
tc_status orient_impl(int64_t n, const OffT* row_ptr, const int32_t* col, OffT* dag_ptr,
                      int32_t* dag_col, int64_t cap, int64_t* m_out, const OrientLayout& L,
                      hipStream_t s) {
  const int grid_rows = grid_for(n, kWavesPerBlock * kGroupsPerWave, 16384);
  // at most n / kLongRow rows can be long
  const int grid_long = (int)std::max<int64_t>(
      1, std::min<int64_t>(2 * device_cu_count(), (n + kLongRow - 1) / kLongRow));
  clear_counter_kernel<<<1, 1, 0, s>>>(L.long_count);
  if (n > 0) {
    if (Order == TC_ORDER_DEGREE)
      degree_kernel<OffT><<<grid_for(n, 256, 8192), 256, 0, s>>>(n, row_ptr, L.deg);
    count_rows_kernel<OffT, Order><<<grid_rows, kBlock, 0, s>>>(n, row_ptr, col, L.deg, L.outdeg,
                                                                L.long_rows, L.long_count);
    count_long_kernel<OffT, Order><<<grid_long, kBlock, 0, s>>>(row_ptr, col, L.deg, L.outdeg,
                                                                L.long_rows, L.long_count);
  }
  hipError_t e = scan_exclusive<OpSum>(n + 1, DegLoad{L.outdeg, n}, OffStore<OffT>{dag_ptr},
                                       L.partial, s);
  if (e != hipSuccess) return check_hip(e, "orient offset scan");
  finalize_kernel<<<1, 1, 0, s>>>(L.partial + scan_num_tiles(n + 1), cap, m_out);
  if (n > 0) {
    fill_rows_kernel<OffT, Order><<<grid_rows, kBlock, 0, s>>>(n, row_ptr, col, L.deg, dag_ptr,
                                                               dag_col, m_out);
    fill_long_kernel<OffT, Order><<<grid_long, kBlock, 0, s>>>(
        row_ptr, col, L.deg, dag_ptr, dag_col, L.long_rows, L.long_count, m_out);
  }
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
  if (sym->offset_bytes != 4 && sym->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", sym->offset_bytes);
  if (order != TC_ORDER_DEGREE && order != TC_ORDER_ID)
    return fail(TC_ERR_INVALID_ARG, "unknown order %d", order);
  tc_status st;
  if (workspace_query(ws, ws_bytes, carve_orient(nullptr, n).bytes, &st)) return st;
  if (!sym->row_ptr || !dag_row_ptr || !m_out || (dag_col_capacity > 0 && !dag_col))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const OrientLayout L = carve_orient(ws, n);
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
