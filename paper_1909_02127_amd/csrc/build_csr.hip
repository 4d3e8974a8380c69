// build_csr.hip - tc_build_csr: raw pairs -> symmetric, deduplicated, self-loop-free CSR.
//
// The problem statement (Sec. II-A) makes G undirected and unlabeled, so (u,v)
// and (v,u) are one edge; Def. 2's injective mapping leaves self-loops out of
// every match.  The graph is stored as CSR (Sec. III-B).
//
// Device pipeline (all on the caller's stream, no host synchronisation):
//   1. make_keys: each pair {a,b}, a != b, emits the packed keys (a<<cb | b) and
//      (b<<cb | a), cb = bits of an id; self-loops and bad pairs emit a sentinel
//      that sorts last; an out-of-range id raises a device error flag.
//   2. LSD radix sort of the 2*num_pairs keys over their 2*cb significant bits,
//      8 bits per pass: per-tile digit histograms, one scan over the
//      digit-major histogram table, and a stable scatter that sorts each tile by
//      digit in LDS (in-tile ranks from 8 wave ballots per key, each wave on its
//      own quarter of the tile) and then writes every digit's run to
//      consecutive addresses.
//   3. One scan over "first of its run" flags drops duplicates and sentinels,
//      writes col, and records the first position of every non-empty row.
//   4. A suffix-minimum scan turns the row starts into row_ptr (empty rows take
//      the next row's start), in int32 or int64 offsets.
//   5. A finalize step reports 2m, or -status with an all-zero row_ptr.
#include "tc_device.h"
#include "tc_host.h"
#include "tc_scan.h"

namespace tc {
namespace {

constexpr int kRadixBlock = 256;
constexpr int kRadixItems = 16;
constexpr int64_t kRadixTile = (int64_t)kRadixBlock * kRadixItems;
constexpr uint64_t kSentinel = ~0ull;

int id_bits(int64_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

// One workgroup per radix tile: its kRadixTile / 2 pairs give the tile's keys,
// whose first-pass digits (key & mask0) are counted into the first pass's tile
// histogram (digit-major).
__global__ __launch_bounds__(kRadixBlock) void make_keys_kernel(int64_t n, int64_t num_pairs,
                                                                const int32_t* __restrict__ src,
                                                                const int32_t* __restrict__ dst,
                                                                int cb, uint32_t mask0,
                                                                uint64_t* __restrict__ keys,
                                                                uint32_t* __restrict__ hist,
                                                                int64_t num_tiles,
                                                                int32_t* __restrict__ err) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  bool bad = false;
  const int64_t first = (int64_t)blockIdx.x * (kRadixTile / 2);
#pragma unroll 4
  for (int r = 0; r < kRadixItems / 2; ++r) {
    const int64_t i = first + (int64_t)r * kRadixBlock + threadIdx.x;
    if (i >= num_pairs) break;
    int64_t a = src[i], b = dst[i];
    uint64_t k0 = kSentinel, k1 = kSentinel;
    if (a < 0 || a >= n || b < 0 || b >= n) {
      bad = true;
    } else if (a != b) {
      k0 = ((uint64_t)a << cb) | (uint64_t)b;
      k1 = ((uint64_t)b << cb) | (uint64_t)a;
    }
    keys[2 * i] = k0;
    keys[2 * i + 1] = k1;
    atomicAdd(&h[(uint32_t)k0 & mask0], 1u);
    atomicAdd(&h[(uint32_t)k1 & mask0], 1u);
  }
  if (ballot(bad) != 0 && lane_id() == 0) atomicOr(err, 1);
  __syncthreads();
  hist[(int64_t)threadIdx.x * num_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRadixBlock) void radix_hist_kernel(const uint64_t* __restrict__ keys,
                                                                 int64_t nk, int shift,
                                                                 uint32_t mask,
                                                                 uint32_t* __restrict__ hist,
                                                                 int64_t num_tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
  for (int r = 0; r < kRadixItems; ++r) {
    int64_t i = base + (int64_t)r * kRadixBlock + threadIdx.x;
    if (i < nk) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * num_tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: keys of equal digit keep their input order.  Each
// wave ranks its own contiguous quarter of the tile, 64 keys per round (peers of
// equal digit from 8 ballots, a per-wave running count per digit), so the only
// workgroup barriers are the few between the phases.  The tile is then sorted by
// digit in LDS and written so that each digit's run lands at consecutive global
// addresses (coalesced stores).
__global__ __launch_bounds__(kRadixBlock) void radix_scatter_kernel(
    const uint64_t* __restrict__ in, uint64_t* __restrict__ out, int64_t nk, int shift, int bits,
    const uint32_t* __restrict__ offsets, int64_t num_tiles) {
  constexpr int kWaves = kRadixBlock / kWave;
  constexpr int kPerWave = kRadixItems * kWave;
  __shared__ uint64_t lkeys[kRadixTile];
  __shared__ uint32_t gbase[256];        // global start of this tile's run of each digit
  __shared__ uint32_t lstart[256];       // start of each digit's run inside the tile
  __shared__ uint32_t wcnt[kWaves][256]; // per-wave digit counts, then per-wave starts
  __shared__ uint32_t wave_tot[kWaves];
  const int t = threadIdx.x;
  const int wave = t / kWave;
  const int lane = lane_id();
  const uint32_t mask = (1u << bits) - 1u;
  const int64_t tile = (int64_t)blockIdx.x * kRadixTile;
  const int valid_n = (int)(nk - tile < kRadixTile ? nk - tile : kRadixTile);
  gbase[t] = offsets[(int64_t)t * num_tiles + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const int wbase = wave * kPerWave;
  uint64_t k[kRadixItems];
  uint32_t rk[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int i = wbase + r * kWave + lane;
    k[r] = i < valid_n ? in[tile + i] : 0;
  }
  // rank of every key among the equal-digit keys before it in this wave's quarter
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const bool ok = wbase + r * kWave + lane < valid_n;
    const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
    uint64_t peers = ballot(ok);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = rank_below(peers);
    const uint32_t before = wcnt[wave][d];
    rk[r] = before + rank;
    wave_sync();
    if (ok && rank == 0) wcnt[wave][d] = before + popc(peers);
    wave_sync();
  }
  __syncthreads();
  // digit t: start of each wave's run inside the digit, and the digit's total
  uint32_t tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t c = wcnt[w][t];
    wcnt[w][t] = tot;
    tot += c;
  }
  {
    uint32_t x = tot;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, kWave);
      if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wave_tot[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wave_tot[w];
    lstart[t] = before + x - tot;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    if (wbase + r * kWave + lane < valid_n) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
      lkeys[lstart[d] + wcnt[wave][d] + rk[r]] = k[r];
    }
  }
  __syncthreads();
  // coalesced write-out of the digit-sorted tile
  for (int j = t; j < valid_n; j += kRadixBlock) {
    const uint64_t key = lkeys[j];
    const uint32_t d = (uint32_t)(key >> shift) & mask;
    out[gbase[d] + (uint32_t)j - lstart[d]] = key;
  }
}

struct HistLoad {
  const uint32_t* hist;
  __device__ int64_t operator()(int64_t i) const { return hist[i]; }
};
struct HistStore {
  uint32_t* hist;
  __device__ void operator()(int64_t i, int64_t p) const { hist[i] = (uint32_t)p; }
};

struct RunFlag {
  const uint64_t* keys;
  __device__ __forceinline__ bool operator()(int64_t i) const {
    const uint64_t k = keys[i];
    return k != kSentinel && (i == 0 || keys[i - 1] != k);
  }
};
struct DedupLoad {
  RunFlag flag;
  __device__ int64_t operator()(int64_t i) const { return flag(i) ? 1 : 0; }
};
struct DedupStore {
  RunFlag flag;
  int cb;
  int32_t* col;
  int64_t cap;
  int64_t* start;
  __device__ void operator()(int64_t i, int64_t pos) const {
    if (!flag(i)) return;
    const uint64_t k = flag.keys[i];
    const uint64_t row = k >> cb;
    if (pos < cap) col[pos] = (int32_t)(k & ((1ull << cb) - 1ull));
    if (i == 0 || (flag.keys[i - 1] >> cb) != row) start[row] = pos;
  }
};

__global__ void fill_i64_kernel(int64_t* p, int64_t len, int64_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = v;
}

__global__ void clear_i32_kernel(int32_t* p) { *p = 0; }

// start[n] = number of distinct entries (total of the dedup scan).
__global__ void set_total_kernel(int64_t* start, int64_t n, const int64_t* dedup_total) {
  start[n] = *dedup_total;
}

// Row offsets: row_ptr[r] = min(start[r..n]) via an exclusive min-scan over reversed rows.
struct SuffixLoad {
  const int64_t* start;
  int64_t n;
  __device__ int64_t operator()(int64_t i) const { return start[n - i]; }
};
template <typename OffT>
struct SuffixStore {
  const int64_t* start;
  int64_t n;
  OffT* row_ptr;
  __device__ void operator()(int64_t i, int64_t exc) const {
    const int64_t s = start[n - i];
    row_ptr[n - i] = (OffT)(s < exc ? s : exc);
  }
};

__global__ void finalize_kernel(const int32_t* err, const int64_t* total, int64_t cap,
                                int64_t* nnz_out) {
  int64_t r = *total;
  if (*err) r = -(int64_t)TC_ERR_ID_OUT_OF_RANGE;
  else if (r > cap) r = -(int64_t)TC_ERR_CAPACITY;
  *nnz_out = r;
}

template <typename OffT>
__global__ void zero_on_error_kernel(OffT* row_ptr, int64_t len, const int64_t* nnz_out) {
  if (*nnz_out >= 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
    row_ptr[i] = 0;
}

struct BuildLayout {
  uint64_t* keys_a;
  uint64_t* keys_b;
  uint32_t* hist;
  int64_t* partial_a;
  int64_t* partial_b;
  int64_t* start;
  int32_t* err;
  size_t bytes;
};

BuildLayout carve_build(void* ws, int64_t n, int64_t num_pairs) {
  const int64_t nk = 2 * num_pairs;
  const int64_t tiles = (nk + kRadixTile - 1) / kRadixTile;
  int64_t pa = scan_partial_len(256 * tiles);
  if (scan_partial_len(n + 1) > pa) pa = scan_partial_len(n + 1);
  Carver c(ws);
  BuildLayout L;
  L.keys_a = c.take<uint64_t>(nk);
  L.keys_b = c.take<uint64_t>(nk);
  L.hist = c.take<uint32_t>(256 * tiles);
  L.partial_a = c.take<int64_t>(pa);
  L.partial_b = c.take<int64_t>(scan_partial_len(nk));
  L.start = c.take<int64_t>(n + 1);
  L.err = c.take<int32_t>(1);
  L.bytes = c.used();
  return L;
}

template <typename OffT>
tc_status build_impl(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
                     OffT* row_ptr, int32_t* col, int64_t cap, int64_t* nnz_out,
                     const BuildLayout& L, hipStream_t s) {
  const int64_t nk = 2 * num_pairs;
  const int cb = id_bits(n);
  const int key_bits = 2 * cb;
  const int64_t tiles = (nk + kRadixTile - 1) / kRadixTile;

  clear_i32_kernel<<<1, 1, 0, s>>>(L.err);
  if (num_pairs > 0) {
    const uint32_t mask0 = (1u << (key_bits < 8 ? key_bits : 8)) - 1u;
    make_keys_kernel<<<(unsigned)tiles, kRadixBlock, 0, s>>>(n, num_pairs, src, dst, cb, mask0,
                                                            L.keys_a, L.hist, tiles, L.err);
  }
  uint64_t* in = L.keys_a;
  uint64_t* out = L.keys_b;
  if (nk > 0) {
    for (int shift = 0; shift < key_bits; shift += 8) {
      const int bits = key_bits - shift < 8 ? key_bits - shift : 8;
      // the first pass's tile histograms come from make_keys
      if (shift > 0)
        radix_hist_kernel<<<(unsigned)tiles, kRadixBlock, 0, s>>>(in, nk, shift, (1u << bits) - 1u,
                                                                 L.hist, tiles);
      hipError_t e = scan_exclusive<OpSum>(256 * tiles, HistLoad{L.hist}, HistStore{L.hist},
                                           L.partial_a, s);
      if (e != hipSuccess) return check_hip(e, "radix digit scan");
      radix_scatter_kernel<<<(unsigned)tiles, kRadixBlock, 0, s>>>(in, out, nk, shift, bits,
                                                                  L.hist, tiles);
      uint64_t* t = in;
      in = out;
      out = t;
    }
  }
  fill_i64_kernel<<<grid_for(n + 1, 256, 4096), 256, 0, s>>>(L.start, n + 1, INT64_MAX);
  RunFlag flag{in};
  hipError_t e = scan_exclusive<OpSum>(nk, DedupLoad{flag}, DedupStore{flag, cb, col, cap, L.start},
                                       L.partial_b, s);
  if (e != hipSuccess) return check_hip(e, "dedup scan");
  const int64_t* dedup_total = L.partial_b + scan_num_tiles(nk);
  set_total_kernel<<<1, 1, 0, s>>>(L.start, n, dedup_total);
  e = scan_exclusive<OpMin>(n + 1, SuffixLoad{L.start, n}, SuffixStore<OffT>{L.start, n, row_ptr},
                            L.partial_a, s);
  if (e != hipSuccess) return check_hip(e, "row offset scan");
  finalize_kernel<<<1, 1, 0, s>>>(L.err, dedup_total, cap, nnz_out);
  zero_on_error_kernel<OffT><<<grid_for(n + 1, 256, 4096), 256, 0, s>>>(row_ptr, n + 1, nnz_out);
  return check_hip(hipGetLastError(), "tc_build_csr launch");
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_build_csr(int64_t n, int64_t num_pairs, const int32_t* src,
                                  const int32_t* dst, int32_t offset_bytes, void* row_ptr,
                                  int32_t* col, int64_t col_capacity, int64_t* nnz_out, void* ws,
                                  size_t* ws_bytes, void* stream) {
  using namespace tc;
  if (n < 0 || num_pairs < 0 || col_capacity < 0)
    return fail(TC_ERR_INVALID_ARG, "negative size (n=%lld num_pairs=%lld capacity=%lld)",
                (long long)n, (long long)num_pairs, (long long)col_capacity);
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (num_pairs > INT32_MAX)
    return fail(TC_ERR_UNSUPPORTED, "num_pairs=%lld exceeds 2^31-1", (long long)num_pairs);
  if (offset_bytes != 4 && offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", offset_bytes);
  if (offset_bytes == 4 && 2 * num_pairs > INT32_MAX)
    return fail(TC_ERR_UNSUPPORTED, "int32 offsets cannot hold 2*num_pairs=%lld entries",
                (long long)(2 * num_pairs));
  const BuildLayout need = carve_build(nullptr, n, num_pairs);
  tc_status st;
  if (workspace_query(ws, ws_bytes, need.bytes, &st)) return st;
  if (!row_ptr || !nnz_out || (num_pairs > 0 && (!src || !dst)) || (col_capacity > 0 && !col))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const BuildLayout L = carve_build(ws, n, num_pairs);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (offset_bytes == 4)
    st = build_impl<int32_t>(n, num_pairs, src, dst, static_cast<int32_t*>(row_ptr), col,
                             col_capacity, nnz_out, L, s);
  else
    st = build_impl<int64_t>(n, num_pairs, src, dst, static_cast<int64_t*>(row_ptr), col,
                             col_capacity, nnz_out, L, s);
  return st == TC_OK ? ok() : st;
}
