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
//   2. LSD radix sort of the 2*num_pairs keys over their 2*cb significant bits
//      in ceil(2*cb / 8) passes of at most 8 bits: per-tile digit histograms,
//      one scan over the digit-major histogram table, and a stable scatter that
//      sorts each tile by digit in LDS (in-tile ranks from one wave ballot per
//      digit bit, each wave on its own quarter of the tile) and then writes
//      every digit's run to consecutive addresses.
//   3. Dedup: a key is kept when it is no sentinel and differs from the key
//      before it.  One pass counts the kept keys of every tile (ballots), the
//      tile counts are scanned, and a second pass writes col at the kept keys'
//      ranks and records the first position of every non-empty row.
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
constexpr int kMaxDigitBits = 8;
constexpr int kMaxDigits = 1 << kMaxDigitBits;
static_assert(kMaxDigits == kRadixBlock, "one digit per thread in the scatter");
constexpr uint64_t kSentinel = ~0ull;

int id_bits(int64_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

// The radix passes over key_bits bits: as few as digits of at most
// kMaxDigitBits allow, with the bits spread evenly (earlier passes take the
// remainder).
struct RadixPlan {
  int passes;
  int key_bits;
  int bits_of(int p) const { return key_bits / passes + (p < key_bits % passes ? 1 : 0); }
  int max_bits() const { return bits_of(0); }
};

RadixPlan radix_plan(int64_t n) {
  const int key_bits = 2 * id_bits(n);
  return RadixPlan{(key_bits + kMaxDigitBits - 1) / kMaxDigitBits, key_bits};
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
  __shared__ uint32_t h[kMaxDigits];
  const int digits = (int)mask0 + 1;
  for (int d = threadIdx.x; d < digits; d += kRadixBlock) h[d] = 0;
  __syncthreads();
  bool bad = false;
  // the tile's pairs, all loads in flight together (clamped to the last pair)
  constexpr int kPairs = kRadixItems / 2;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t first = tile * (kRadixTile / 2);
  const int valid = (int)(num_pairs - first < kRadixTile / 2 ? num_pairs - first : kRadixTile / 2);
  int32_t pa[kPairs], pb[kPairs];
#pragma unroll
  for (int r = 0; r < kPairs; ++r) {
    const int j = r * kRadixBlock + (int)threadIdx.x;
    const int64_t i = first + (j < valid ? j : valid - 1);
    pa[r] = src[i];
    pb[r] = dst[i];
  }
#pragma unroll
  for (int r = 0; r < kPairs; ++r) {
    const int j = r * kRadixBlock + (int)threadIdx.x;
    if (j >= valid) continue;
    const int64_t i = first + j;
    const int64_t a = pa[r], b = pb[r];
    uint64_t k0 = kSentinel, k1 = kSentinel;
    if (a < 0 || a >= n || b < 0 || b >= n) {
      bad = true;
    } else if (a != b) {
      k0 = ((uint64_t)a << cb) | (uint64_t)b;
      k1 = ((uint64_t)b << cb) | (uint64_t)a;
    }
    // both keys of the pair in one 16-byte store (keys is 16-byte aligned)
    reinterpret_cast<ulonglong2*>(keys)[i] = make_ulonglong2(k0, k1);
    atomicAdd(&h[(uint32_t)k0 & mask0], 1u);
    atomicAdd(&h[(uint32_t)k1 & mask0], 1u);
  }
  if (ballot(bad) != 0 && lane_id() == 0) atomicOr(err, 1);
  __syncthreads();
  for (int d = threadIdx.x; d < digits; d += kRadixBlock)
    hist[(int64_t)d * num_tiles + tile] = h[d];
}

__global__ __launch_bounds__(kRadixBlock) void radix_hist_kernel(const uint64_t* __restrict__ keys,
                                                                 int64_t nk, int shift,
                                                                 uint32_t mask,
                                                                 uint32_t* __restrict__ hist,
                                                                 int64_t num_tiles) {
  __shared__ uint32_t h[kMaxDigits];
  const int digits = (int)mask + 1;
  for (int d = threadIdx.x; d < digits; d += kRadixBlock) h[d] = 0;
  __syncthreads();
  // the tile's keys, all loads in flight together (clamped to the last key)
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t base = tile * kRadixTile;
  const int valid = (int)(nk - base < kRadixTile ? nk - base : kRadixTile);
  uint64_t k[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int j = r * kRadixBlock + (int)threadIdx.x;
    k[r] = keys[base + (j < valid ? j : valid - 1)];
  }
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r)
    if (r * kRadixBlock + (int)threadIdx.x < valid)
      atomicAdd(&h[(uint32_t)(k[r] >> shift) & mask], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < digits; d += kRadixBlock)
    hist[(int64_t)d * num_tiles + tile] = h[d];
}

// Stable scatter of one tile: keys of equal digit keep their input order.  Each
// wave ranks its own contiguous quarter of the tile, 64 keys per round (peers of
// equal digit from one ballot per digit bit, a per-wave running count per
// digit), so the only
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
  const int64_t tile_id = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t tile = tile_id * kRadixTile;
  const int valid_n = (int)(nk - tile < kRadixTile ? nk - tile : kRadixTile);
  // the histogram table holds rows for the pass's digits only
  if (t < (1 << bits)) gbase[t] = offsets[(int64_t)t * num_tiles + tile_id];
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
    const uint32_t x = (uint32_t)wave_inclusive_sum32((int32_t)tot);  // tot <= kRadixTile
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

// Dedup over the sorted keys, one wave per kDedupRun consecutive keys: a key is
// kept when it is no sentinel and differs from the key before it.
constexpr int kDedupBlock = 256;
constexpr int kDedupItems = 16;
constexpr int kDedupRun = kDedupItems * kWave;
constexpr int64_t kDedupTile = (int64_t)kDedupBlock * kDedupItems;

// Lane l gets x of lane l - 1 and lane 0 gets `first`: a whole-wave DPP shift
// (wave_shr:1, control 0x138) on each 32-bit half, with no LDS round trip.  A
// lane without a source keeps `old` (bound_ctrl off).  Called by the whole wave.
__device__ __forceinline__ uint64_t wave_shift_up1_u64(uint64_t x, uint64_t first) {
  constexpr int kWaveShr1 = 0x138;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(
      (int)(uint32_t)first, (int)(uint32_t)x, kWaveShr1, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
      (int)(uint32_t)(first >> 32), (int)(uint32_t)(x >> 32), kWaveShr1, 0xf, 0xf, false);
  return ((uint64_t)hi << 32) | lo;
}

// Loads the wave's run and returns the kept-key mask of every round.
__device__ __forceinline__ void dedup_load(const uint64_t* __restrict__ keys, int64_t nk,
                                           int64_t base, uint64_t (&k)[kDedupItems],
                                           uint64_t (&keep)[kDedupItems]) {
  const int lane = lane_id();
#pragma unroll
  for (int r = 0; r < kDedupItems; ++r) {
    const int64_t i = base + (int64_t)r * kWave + lane;
    k[r] = i < nk ? keys[i] : kSentinel;
  }
  // the key before lane 0 of the first round (none for the first key)
  uint64_t prev = base > 0 && base <= nk ? keys[base - 1] : kSentinel;
  const bool first_key = base == 0;
#pragma unroll
  for (int r = 0; r < kDedupItems; ++r) {
    const uint64_t p = wave_shift_up1_u64(k[r], prev);
    const bool head = r == 0 && lane == 0 && first_key;
    keep[r] = ballot(k[r] != kSentinel && (head || p != k[r]));
    prev = (uint64_t)read_lane64((int64_t)k[r], kWave - 1);
  }
}

__global__ __launch_bounds__(kDedupBlock) void dedup_count_kernel(const uint64_t* __restrict__ keys,
                                                                  int64_t nk,
                                                                  int64_t* __restrict__ partial) {
  __shared__ uint32_t wave_cnt[kDedupBlock / kWave];
  const int wave = threadIdx.x / kWave;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t base = tile * kDedupTile + (int64_t)wave * kDedupRun;
  uint64_t k[kDedupItems], keep[kDedupItems];
  dedup_load(keys, nk, base, k, keep);
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < kDedupItems; ++r) c += popc(keep[r]);
  if (lane_id() == 0) wave_cnt[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kDedupBlock / kWave; ++w) tot += wave_cnt[w];
    partial[tile] = tot;
  }
}

// partial[] holds the exclusive scan of the tile counts.  Kept keys go to col at
// their rank (while it is below cap), and the first kept key of each row gives
// start[row].
__global__ __launch_bounds__(kDedupBlock) void dedup_write_kernel(
    const uint64_t* __restrict__ keys, int64_t nk, int cb, const int64_t* __restrict__ partial,
    int32_t* __restrict__ col, int64_t cap, int64_t* __restrict__ start) {
  __shared__ uint32_t wave_cnt[kDedupBlock / kWave];
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t base = tile * kDedupTile + (int64_t)wave * kDedupRun;
  uint64_t k[kDedupItems], keep[kDedupItems];
  dedup_load(keys, nk, base, k, keep);
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < kDedupItems; ++r) c += popc(keep[r]);
  if (lane == 0) wave_cnt[wave] = c;
  __syncthreads();
  int64_t pos = partial[tile];
  for (int w = 0; w < wave; ++w) pos += wave_cnt[w];
  // the row of the key before the wave's run (a kept key whose row differs
  // from its predecessor's starts that row)
  uint64_t prev_row = base > 0 && base <= nk ? keys[base - 1] >> cb : ~0ull;
  const uint64_t id_mask = (1ull << cb) - 1ull;
#pragma unroll
  for (int r = 0; r < kDedupItems; ++r) {
    const uint64_t row = k[r] >> cb;
    const uint64_t p = wave_shift_up1_u64(row, prev_row);
    if ((keep[r] >> lane) & 1u) {
      const int64_t at = pos + rank_below(keep[r]);
      if (at < cap) col[at] = (int32_t)(k[r] & id_mask);
      if (p != row) start[row] = at;
    }
    pos += popc(keep[r]);
    prev_row = (uint64_t)read_lane64((int64_t)row, kWave - 1);
  }
}

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
  const int64_t digits = (int64_t)1 << radix_plan(n).max_bits();
  int64_t pa = scan_partial_len(digits * tiles);
  if (scan_partial_len(n + 1) > pa) pa = scan_partial_len(n + 1);
  Carver c(ws);
  BuildLayout L;
  L.keys_a = c.take<uint64_t>(nk);
  L.keys_b = c.take<uint64_t>(nk);
  L.hist = c.take<uint32_t>(digits * tiles);
  L.partial_a = c.take<int64_t>(pa);
  L.partial_b = c.take<int64_t>((nk + kDedupTile - 1) / kDedupTile + 1);
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
  const RadixPlan plan = radix_plan(n);
  const int64_t tiles = (nk + kRadixTile - 1) / kRadixTile;

  clear_i32_kernel<<<1, 1, 0, s>>>(L.err);
  if (num_pairs > 0) {
    const uint32_t mask0 = (1u << plan.bits_of(0)) - 1u;
    make_keys_kernel<<<(unsigned)tiles, kRadixBlock, 0, s>>>(n, num_pairs, src, dst, cb, mask0,
                                                            L.keys_a, L.hist, tiles, L.err);
  }
  uint64_t* in = L.keys_a;
  uint64_t* out = L.keys_b;
  if (nk > 0) {
    int shift = 0;
    for (int pass = 0; pass < plan.passes; ++pass) {
      const int bits = plan.bits_of(pass);
      const int64_t digits = (int64_t)1 << bits;
      // the first pass's tile histograms come from make_keys
      if (pass > 0)
        radix_hist_kernel<<<(unsigned)tiles, kRadixBlock, 0, s>>>(in, nk, shift, (1u << bits) - 1u,
                                                                 L.hist, tiles);
      hipError_t e = scan_exclusive<OpSum>(digits * tiles, HistLoad{L.hist}, HistStore{L.hist},
                                           L.partial_a, s);
      if (e != hipSuccess) return check_hip(e, "radix digit scan");
      radix_scatter_kernel<<<(unsigned)tiles, kRadixBlock, 0, s>>>(in, out, nk, shift, bits,
                                                                  L.hist, tiles);
      shift += bits;
      uint64_t* t = in;
      in = out;
      out = t;
    }
  }
  fill_i64_kernel<<<grid_for(n + 1, 256, 4096), 256, 0, s>>>(L.start, n + 1, INT64_MAX);
  const int64_t dtiles = (nk + kDedupTile - 1) / kDedupTile;
  if (dtiles > 0)
    dedup_count_kernel<<<(unsigned)dtiles, kDedupBlock, 0, s>>>(in, nk, L.partial_b);
  scan_partials_kernel<OpSum><<<1, 1024, 0, s>>>(dtiles, L.partial_b);
  if (dtiles > 0)
    dedup_write_kernel<<<(unsigned)dtiles, kDedupBlock, 0, s>>>(in, nk, cb, L.partial_b, col, cap,
                                                                L.start);
  const int64_t* dedup_total = L.partial_b + dtiles;
  set_total_kernel<<<1, 1, 0, s>>>(L.start, n, dedup_total);
  hipError_t e = scan_exclusive<OpMin>(n + 1, SuffixLoad{L.start, n},
                                       SuffixStore<OffT>{L.start, n, row_ptr}, L.partial_a, s);
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
