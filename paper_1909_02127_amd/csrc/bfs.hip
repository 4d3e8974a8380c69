// bfs.hip - the paper's own pipeline, for comparison with the fused count:
// the NE candidate filter and a materialised two-iteration advance.
//
// tc_ne_filter: Alg. 1 filters candidate data vertices by their neighbourhood
// encoding (NE = degree) against the query's; for the triangle every query node
// has degree 2.  Here the filter is iterated (a vertex must keep 2 candidate
// neighbours), which converges to the 2-core; any number of rounds preserves
// every triangle.  Rounds update in place and stop early once a round removes
// nothing (later launches exit at once), so no host synchronisation is needed.
//
// tc_count_bfs: the BFS-style verification of Alg. 1 with its intermediate
// results written out.  Iteration 1 advances every candidate source u to its
// out-neighbours v (the unique mapping order makes the DAG the candidate edges)
// and compacts the partial matches (u, v) that pass the look-ahead filters of
// Sec. III-C (d+(u) >= 2, d+(v) >= 1) and the NE filter.  Iteration 2 advances
// each partial match to every w in N+(v) and keeps the wedge when the stored
// non-tree edge (u, w) exists ("Store_none_tree_connection"; checked by binary
// search in the sorted row of u): the complete matches, compacted into M.  The
// second advance is load-balanced over candidate wedges in fixed tiles: a tile
// finds its first partial match with a 64-way wave search over the prefix sums
// of the frontier's work.
#include "tc_device.h"
#include "tc_host.h"
#include "tc_scan.h"

#include <algorithm>

namespace tc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;
constexpr int kPadded = kTile + kTile / kItems;
constexpr int kChunkRows = 256;  // rows per wave and claim in the frontier pass

__device__ __forceinline__ int padded(int i) { return i + (i >> 4); }

// ---- NE filter ---------------------------------------------------------------

__global__ void ne_init_kernel(int64_t n, uint8_t* __restrict__ keep, int32_t* __restrict__ flags,
                               int32_t rounds) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t v = t; v < n; v += stride) keep[v] = 1;
  for (int64_t r = t; r <= rounds; r += stride) flags[r] = 0;
}

// One round: every surviving vertex with fewer than k surviving neighbours is
// removed.  Skipped when the previous round removed nothing.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void ne_round_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col,
                                                          int32_t k, uint8_t* __restrict__ keep,
                                                          int32_t* __restrict__ flags, int32_t r) {
  if (r > 0 && flags[r - 1] == 0) return;
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
  bool removed = false;
  for (int64_t v = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; v < n; v += waves) {
    if (!keep[v]) continue;
    const int64_t b = row_ptr[v], e = row_ptr[v + 1];
    int64_t alive = 0;
    for (int64_t i = b + lane; i - lane < e && alive < k; i += kWave)
      alive += popc(ballot(i < e && keep[col[i]] != 0));
    if (alive < k) {
      if (lane == 0) keep[v] = 0;
      removed = true;
    }
  }
  if (removed && lane == 0) flags[r] = 1;
}

// stats = {vertices kept, rounds that removed something, converged}.
__global__ __launch_bounds__(kBlock) void ne_finish_kernel(int64_t n, const uint8_t* __restrict__ keep,
                                                           const int32_t* __restrict__ flags,
                                                           int32_t rounds, int64_t* stats) {
  __shared__ int64_t part[kWavesPerBlock];
  int64_t c = 0;
  for (int64_t v = threadIdx.x; v < n; v += kBlock) c += keep[v];
  c = wave_sum(c);
  if (lane_id() == 0) part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t kept = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) kept += part[w];
    int64_t changed = 0;
    for (int r = 0; r < rounds; ++r) changed += flags[r] != 0;
    stats[0] = kept;
    stats[1] = changed;
    stats[2] = rounds == 0 ? 0 : (flags[rounds - 1] == 0);
  }
}

// ---- materialised two-iteration advance ------------------------------------

struct BfsState {
  int64_t frontier;  // partial matches after iteration 1 (may exceed the capacity)
  int64_t matches;   // complete matches (may exceed the match capacity)
  int64_t cursor;    // output rows handed out
  int32_t status;    // 0, or TC_ERR_CAPACITY
  int32_t pad;
};

__global__ void bfs_init_kernel(BfsState* st) {
  st->frontier = 0;
  st->matches = 0;
  st->cursor = 0;
  st->status = 0;
}

__device__ __forceinline__ bool kept(const uint8_t* keep, int64_t v) { return !keep || keep[v]; }

// Iteration 1: a wave claims kChunkRows rows, counts their partial matches
// (u, v), takes that many frontier slots with one atomic, and writes them.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void advance1_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col,
                                                          const uint8_t* __restrict__ keep,
                                                          int64_t cap, int32_t* __restrict__ fu,
                                                          int32_t* __restrict__ fv,
                                                          BfsState* __restrict__ st) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t r0 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * kChunkRows; r0 < n;
       r0 += waves * kChunkRows) {
    const int64_t r1 = r0 + kChunkRows < n ? r0 + kChunkRows : n;
    int64_t count = 0;
    for (int pass = 0; pass < 2; ++pass) {
      int64_t base = 0;
      if (pass == 1) {
        if (count == 0) break;
        if (lane == 0) base = atomicAdd((unsigned long long*)&st->frontier, (unsigned long long)count);
        base = read_lane64(base, 0);
      }
      for (int64_t u = r0; u < r1; ++u) {
        const int64_t b = row_ptr[u], e = row_ptr[u + 1];
        if (e - b < 2 || !kept(keep, u)) continue;  // 2-look-ahead
        for (int64_t i = b + lane; i - lane < e; i += kWave) {
          int32_t v = 0;
          bool ok = false;
          if (i < e) {
            v = col[i];
            ok = kept(keep, v) && row_ptr[v + 1] > row_ptr[v];  // 1-look-ahead
          }
          const uint64_t m = ballot(ok);
          if (pass == 0) {
            count += popc(m);
          } else {
            const int64_t at = base + rank_below(m);
            if (ok && at < cap) {
              fu[at] = (int32_t)u;
              fv[at] = v;
            }
            base += popc(m);
          }
        }
      }
    }
  }
}

__global__ void frontier_check_kernel(int64_t cap, BfsState* st) {
  if (st->frontier > cap) st->status = TC_ERR_CAPACITY;
}

// Work of each partial match: d+(v).
template <typename OffT>
struct WorkLoad {
  const OffT* row_ptr;
  const int32_t* fv;
  const BfsState* st;
  __device__ int64_t operator()(int64_t f) const {
    if (st->status || f >= st->frontier) return 0;
    const int32_t v = fv[f];
    return (int64_t)(row_ptr[v + 1] - row_ptr[v]);
  }
};
struct WorkStore {
  int64_t* pre;
  __device__ void operator()(int64_t f, int64_t p) const { pre[f] = p; }
};

// Largest f in [0, F) with pre[f] <= x (pre strictly increasing, pre[0] = 0 <= x):
// a 64-way search, one gather per level.  Called by a whole wave.
__device__ __forceinline__ int64_t wave_find(const int64_t* __restrict__ pre, int64_t F, int64_t x) {
  const int lane = lane_id();
  int64_t lo = 0, hi = F;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + kWave - 1) / kWave;
    const int64_t idx = lo + (int64_t)lane * step;
    const bool ok = idx < hi && pre[idx] <= x;
    const int64_t c = popc(ballot(ok));  // >= 1: lane 0 probes lo
    const int64_t nlo = lo + (c - 1) * step;
    const int64_t nhi = lo + c * step < hi ? lo + c * step : hi;
    lo = nlo;
    hi = nhi;
  }
  return lo;
}

// Is w in the sorted row [b, e) of col?
__device__ __forceinline__ bool in_row(const int32_t* __restrict__ col, int64_t b, int64_t e,
                                       int32_t w) {
  while (b < e) {
    const int64_t mid = b + ((e - b) >> 1);
    const int32_t x = col[mid];
    if (x < w) b = mid + 1;
    else if (x > w) e = mid;
    else return true;
  }
  return false;
}

// Iteration 2 over tiles of kTile candidate wedges; per tile: find the first
// partial match, mark where each later one starts, give every candidate its
// partial match by a max-scan, check the closing edge, count, and (when asked)
// write the complete matches at slots taken with one atomic per tile.
template <typename OffT>
__global__ __launch_bounds__(kBlock) void advance2_kernel(
    const OffT* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const uint8_t* __restrict__ keep, const int32_t* __restrict__ fu, const int32_t* __restrict__ fv,
    const int64_t* __restrict__ pre, const int64_t* __restrict__ total_work, int32_t* __restrict__ out,
    int64_t out_cap, BfsState* __restrict__ st) {
  __shared__ int32_t smark[kPadded];
  __shared__ int32_t wave_tot[kWavesPerBlock];
  __shared__ int64_t f0_s, obase_s;
  if (st->status) return;
  const int64_t F = st->frontier;
  const int64_t W = *total_work;
  const int64_t tiles = (W + kTile - 1) / kTile;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t x0 = t * kTile;
    const int len = (int)(W - x0 < kTile ? W - x0 : kTile);
    if (wave == 0) {
      const int64_t f0 = wave_find(pre, F, x0);
      if (lane == 0) f0_s = f0;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) smark[padded(k * kBlock + tid)] = -1;
    __syncthreads();
    const int64_t f0 = f0_s;
    // partial matches starting inside the tile (work >= 1 each, so at most kTile)
    for (int64_t f = f0 + 1 + tid; f < F; f += kBlock) {
      const int64_t p = pre[f] - x0;
      if (p >= len) break;
      smark[padded((int)p)] = (int32_t)(f - f0);
    }
    __syncthreads();
    int32_t agg = -1;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int32_t mk = smark[padded(tid * kItems + k)];
      agg = agg > mk ? agg : mk;
    }
    int32_t inc = wave_inclusive_max32(agg);
    if (lane == kWave - 1) wave_tot[wave] = inc;
    __syncthreads();
    int32_t start = __shfl_up(inc, 1, kWave);
    if (lane == 0) start = -1;
    for (int w = 0; w < wave; ++w) start = start > wave_tot[w] ? start : wave_tot[w];
    start = start > 0 ? start : 0;  // relative index of the partial match of the first item
    // pass 1: the closing-edge check
    uint32_t hit = 0;
    int32_t cur = start;
    for (int k = 0; k < kItems; ++k) {
      const int i = tid * kItems + k;
      const int32_t mk = smark[padded(i)];
      cur = cur > mk ? cur : mk;
      if (i >= len) break;
      const int64_t f = f0 + cur;
      const int32_t u = fu[f], v = fv[f];
      const int32_t w = col[(int64_t)row_ptr[v] + (x0 + i - pre[f])];
      if (kept(keep, w) && in_row(col, row_ptr[u], row_ptr[u + 1], w)) hit |= 1u << k;
    }
    const int32_t mine = (int32_t)popc((uint64_t)hit);
    const int32_t winc = wave_inclusive_sum32(mine);
    if (lane == kWave - 1) wave_tot[wave] = winc;
    __syncthreads();
    int32_t before = winc - mine, kept_tile = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      if (w < wave) before += wave_tot[w];
      kept_tile += wave_tot[w];
    }
    if (tid == 0 && kept_tile) {
      atomicAdd((unsigned long long*)&st->matches, (unsigned long long)kept_tile);
      obase_s = out ? (int64_t)atomicAdd((unsigned long long*)&st->cursor,
                                         (unsigned long long)kept_tile)
                    : 0;
    }
    __syncthreads();
    // pass 2: write the complete matches (u, v, w)
    if (out && hit) {
      int64_t row = obase_s + before;
      cur = start;
      for (int k = 0; k < kItems; ++k) {
        const int i = tid * kItems + k;
        const int32_t mk = smark[padded(i)];
        cur = cur > mk ? cur : mk;
        if (!((hit >> k) & 1u)) continue;
        const int64_t f = f0 + cur;
        const int32_t u = fu[f], v = fv[f];
        const int32_t w = col[(int64_t)row_ptr[v] + (x0 + i - pre[f])];
        if (row < out_cap) {
          out[3 * row + 0] = u;
          out[3 * row + 1] = v;
          out[3 * row + 2] = w;
        }
        ++row;
      }
    }
    __syncthreads();
  }
}

// stats = {frontier, candidate wedges, matches, status}; total = matches.
__global__ void bfs_finish_kernel(const BfsState* st, const int64_t* total_work, int64_t out_cap,
                                  bool has_out, int64_t* stats, uint64_t* total) {
  const int64_t status = st->status ? st->status
                                    : ((has_out && st->matches > out_cap) ? TC_ERR_CAPACITY : 0);
  stats[0] = st->frontier;
  stats[1] = st->status ? 0 : *total_work;
  stats[2] = st->status ? 0 : st->matches;
  stats[3] = status;
  if (total) *total = st->status ? 0 : (uint64_t)st->matches;
}

struct BfsLayout {
  BfsState* st;
  int32_t* fu;
  int32_t* fv;
  int64_t* pre;
  int64_t* partial;
  size_t bytes;
};

BfsLayout carve_bfs(void* ws, int64_t cap) {
  Carver c(ws);
  BfsLayout L;
  L.st = c.take<BfsState>(1);
  L.fu = c.take<int32_t>(cap);
  L.fv = c.take<int32_t>(cap);
  L.pre = c.take<int64_t>(cap);
  L.partial = c.take<int64_t>(scan_partial_len(cap));
  L.bytes = c.used();
  return L;
}

template <typename OffT>
tc_status bfs_impl(int64_t n, const OffT* row_ptr, const int32_t* col, const uint8_t* keep,
                   int64_t cap, int32_t* out, int64_t out_cap, int64_t* stats, uint64_t* total,
                   const BfsLayout& L, hipStream_t s) {
  const int grid = 4 * device_cu_count();
  bfs_init_kernel<<<1, 1, 0, s>>>(L.st);
  if (n > 0)
    advance1_kernel<OffT><<<grid_for(n, kWavesPerBlock * kChunkRows, grid), kBlock, 0, s>>>(
        n, row_ptr, col, keep, cap, L.fu, L.fv, L.st);
  frontier_check_kernel<<<1, 1, 0, s>>>(cap, L.st);
  hipError_t e = scan_exclusive<OpSum>(cap, WorkLoad<OffT>{row_ptr, L.fv, L.st}, WorkStore{L.pre},
                                       L.partial, s);
  if (e != hipSuccess) return check_hip(e, "frontier work scan");
  const int64_t* total_work = L.partial + scan_num_tiles(cap);
  advance2_kernel<OffT><<<grid, kBlock, 0, s>>>(row_ptr, col, keep, L.fu, L.fv, L.pre, total_work,
                                                out, out_cap, L.st);
  bfs_finish_kernel<<<1, 1, 0, s>>>(L.st, total_work, out_cap, out != nullptr, stats, total);
  return check_hip(hipGetLastError(), "tc_count_bfs launch");
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_ne_filter(const tc_csr* sym, int32_t min_degree, int32_t max_rounds,
                                  uint8_t* keep, int64_t* stats_out, void* ws, size_t* ws_bytes,
                                  void* stream) {
  using namespace tc;
  if (!sym) return fail(TC_ERR_INVALID_ARG, "sym is NULL");
  const int64_t n = sym->n;
  if (n < 0) return fail(TC_ERR_INVALID_ARG, "negative n");
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (sym->offset_bytes != 4 && sym->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", sym->offset_bytes);
  if (min_degree < 0 || max_rounds < 0 || max_rounds > 4096)
    return fail(TC_ERR_INVALID_ARG, "min_degree must be >= 0 and max_rounds in [0, 4096]");
  Carver c0(nullptr);
  (void)c0.take<int32_t>(max_rounds + 1);
  tc_status st;
  if (workspace_query(ws, ws_bytes, c0.used(), &st)) return st;
  if (!sym->row_ptr || !stats_out || (n > 0 && !keep))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  Carver c(ws);
  int32_t* flags = c.take<int32_t>(max_rounds + 1);
  hipStream_t s = static_cast<hipStream_t>(stream);
  ne_init_kernel<<<grid_for(std::max<int64_t>(n, max_rounds + 1), 256, 4096), 256, 0, s>>>(
      n, keep, flags, max_rounds);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 3) / 4, 4 * device_cu_count()));
  for (int32_t r = 0; r < max_rounds && n > 0; ++r) {
    if (sym->offset_bytes == 4)
      ne_round_kernel<int32_t><<<grid, kBlock, 0, s>>>(
          n, static_cast<const int32_t*>(sym->row_ptr), sym->col, min_degree, keep, flags, r);
    else
      ne_round_kernel<int64_t><<<grid, kBlock, 0, s>>>(
          n, static_cast<const int64_t*>(sym->row_ptr), sym->col, min_degree, keep, flags, r);
  }
  ne_finish_kernel<<<1, kBlock, 0, s>>>(n, keep, flags, max_rounds, stats_out);
  st = check_hip(hipGetLastError(), "tc_ne_filter launch");
  return st == TC_OK ? ok() : st;
}

extern "C" tc_status tc_count_bfs(const tc_csr* dag, const uint8_t* keep, int64_t frontier_capacity,
                                  int32_t* matches, int64_t match_capacity, int64_t* stats_out,
                                  uint64_t* total, void* ws, size_t* ws_bytes, void* stream) {
  using namespace tc;
  if (!dag) return fail(TC_ERR_INVALID_ARG, "dag is NULL");
  const int64_t n = dag->n;
  if (n < 0 || frontier_capacity < 0 || match_capacity < 0)
    return fail(TC_ERR_INVALID_ARG, "negative size");
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (frontier_capacity > ((int64_t)1 << 34))
    return fail(TC_ERR_UNSUPPORTED, "frontier_capacity beyond 2^34");
  if (dag->offset_bytes != 4 && dag->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", dag->offset_bytes);
  tc_status st;
  if (workspace_query(ws, ws_bytes, carve_bfs(nullptr, frontier_capacity).bytes, &st)) return st;
  if (!dag->row_ptr || !stats_out || (matches == nullptr && match_capacity > 0))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const BfsLayout L = carve_bfs(ws, frontier_capacity);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dag->offset_bytes == 4)
    st = bfs_impl<int32_t>(n, static_cast<const int32_t*>(dag->row_ptr), dag->col, keep,
                           frontier_capacity, matches, match_capacity, stats_out, total, L, s);
  else
    st = bfs_impl<int64_t>(n, static_cast<const int64_t*>(dag->row_ptr), dag->col, keep,
                           frontier_capacity, matches, match_capacity, stats_out, total, L, s);
  return st == TC_OK ? ok() : st;
}
