// count.hip - tc_count / tc_count_per_vertex: all-source wedge advance + closing-edge filter.
//
// Alg. 1 verifies the triangle query in |Q|-1 = 2 BFS iterations from every
// candidate source: the first advance u -> v, the second v -> w, and a match
// needs the stored non-tree query edge (u1,u3), i.e. w in N+(u)
// ("Store_none_tree_connection").  Here the two iterations are fused into one
// pass that never materialises partial results: for each source u the group
// (one workgroup, or one wave for small sources) stages N+(u) in an LDS table,
// then streams every N+(v), v in N+(u), with coalesced reads and probes each w.
// The count is the number of hits, which equals |M|/|Q| of Alg. 1 because the
// orientation (unique mapping order) makes every triangle appear once.
//
// Pruning (Sec. III-C k-look-ahead): a source with d+(u) < 2 cannot close a
// wedge (2-look-ahead) and is never queued; a middle v with d+(v) = 0 adds no
// work (1-look-ahead).
//
// Probe structure: two-choice cuckoo hashing in LDS (two bit fields of one
// multiplicative hash index the two halves of the table, load <= 0.4), so a
// probe is exactly two LDS reads with no data-dependent loop.  Keys that do not settle
// within kMaxKicks evictions go to a small stash; if the stash overflows the
// group falls back to binary search: it refills the (then unused) slot array
// with N+(u), which is sorted, from global memory.
//
// Load balance: sources are binned by d+(u); sources above the split
// (tc_tune.small_max, default kSmallDefault, at most kSmallMax) are handed out
// largest class first through a global cursor, one workgroup each (its four
// waves take the v's round robin); the rest are handled one wave each, in runs
// whose source ids and row bounds are loaded together.
// N+(u) longer than kChunk is processed in kChunk-sized slices of the table.
//
// Per-vertex counts: t(u) += hits of source u; t(v) += hits of the edge (u,v)
// and t(w) += hits closed at w both gather in the LDS slot counters of v and w
// (when the table holds all of N+(u); split sources add t(v) directly) and are
// flushed once per source; each lane keeps its middle's (u,v) count in a
// register until the batch of 64 middles is done.  Global atomics are at most
// n + 2m rather than one per triangle.
#include "tc_device.h"
#include "tc_hash.h"
#include "tc_host.h"
#include "tc_scan.h"

#include <algorithm>
#include <atomic>
#include <mutex>

namespace tc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kSmallMax = 96;    // largest d+(u) a wave may take alone (tc_tune.small_max cap)
constexpr int kSmallDefault = 80;  // default wave/workgroup split on d+(u)
constexpr int kSideMax = 1024;   // slots per cuckoo half (workgroup mode)
constexpr int kChunk = 816;      // keys per LDS table slice: side_log2(kChunk) <= log2(kSideMax)
constexpr int kSmallSide = 128;  // slots per cuckoo half for kSmallMax keys (load <= 0.4)
constexpr int kStash = 32;
constexpr int kMaxKicks = 48;
constexpr int kUnroll = 4;       // 64-wide loads in flight per wave while streaming N+(v)
constexpr int kShortMax = 128;   // middles with d+(v) < kShortMax may be walked as one concatenation
constexpr int kShortMinLists = 4;  // ... when a batch of 64 middles holds at least this many
constexpr int kWin = 2;          // 64-wide windows per step of that walk
constexpr int32_t kEmpty = -1;
constexpr int32_t kNoKey = -2;  // probe value of an inactive lane: never stored
constexpr int kNumClasses = 8;  // 0..6: workgroup classes by size (largest first), 7: small

// What a count launch produces.
constexpr int kKindTotal = 0;      // the total (and optionally per-graph / per-source sums)
constexpr int kKindPerVertex = 1;  // plus t(v) for every vertex
constexpr int kKindList = 2;       // every triangle as a (u, v, w) row
constexpr int kKindSupport = 3;    // triangles on every oriented edge
constexpr int kKindDirected = 4;   // matches of a query on per-edge codes: arc directions or
                                   // edge labels (weighted hits)
// Kinds that count hits per LDS slot (the (u, w) pairs of a source).
__host__ __device__ constexpr bool counted(int kind) {
  return kind == kKindPerVertex || kind == kKindSupport;
}
// Kinds whose table keeps a word per slot: the hit counters, or (directed) the
// arc directions of the edge (u, key).
__host__ __device__ constexpr bool slot_words(int kind) {
  return counted(kind) || kind == kKindDirected;
}

// Probe modes, fixed per table slice after it is built.
constexpr int kModeCuckoo = 0;  // every key sits in one of its two cuckoo slots
constexpr int kModeStash = 1;   // plus up to kStash keys in the stash
constexpr int kModeSorted = 2;  // stash overflowed: binary search the keys, sorted in the slots
constexpr int kModeGlobal = 3;  // N+(u) too long for a few slices: binary search it in memory
constexpr int64_t kGlobalMin = 4 * 816;  // d+(u) above which a source takes kModeGlobal

__host__ __device__ constexpr int small_bytes_per_wave(bool pv) {
  return (2 * kSmallSide) * 4 * (pv ? 2 : 1) + kStash * 8 + 16;
}
__host__ __device__ constexpr int group_bytes(bool pv) {
  return (2 * kSideMax) * 4 * (pv ? 2 : 1) + kStash * 8 + 16;
}
__host__ __device__ constexpr int smem_bytes(bool pv) {
  return group_bytes(pv) > kWavesPerBlock * small_bytes_per_wave(pv)
             ? group_bytes(pv)
             : kWavesPerBlock * small_bytes_per_wave(pv);
}
// Per-wave scratch of the short-list walk: segment-start markers (+ hit counters).
__host__ __device__ constexpr int seg_bytes_per_wave(bool pv) {
  return kWin * kWave * 4 + (pv ? kWave * 4 : 0);
}
__host__ __device__ constexpr int smem_total(bool pv) {
  return smem_bytes(pv) + kWavesPerBlock * seg_bytes_per_wave(pv);
}

struct WaveScratch {
  int32_t* mark;    // [kWin * kWave] segment starting at each position of the window, or -1
  uint32_t* shits;  // [kWave] hits per segment (per-vertex mode)
};

// Size class of a source by out-degree; -1 when it cannot close a wedge.
// Sources with d+ <= small_max (<= kSmallMax) take the one-wave path.
__device__ __forceinline__ int source_class(int64_t d, int small_max) {
  if (d < 2) return -1;
  if (d <= small_max) return 7;
  if (d <= 128) return 6;
  if (d <= 256) return 5;
  if (d <= 512) return 4;
  if (d <= 1024) return 3;
  if (d <= 2048) return 2;
  if (d <= 4096) return 1;
  return 0;
}

struct CountState {
  int32_t class_count[kNumClasses];
  int32_t class_cursor[kNumClasses];
  int32_t large_cursor;
  int32_t small_cursor;
  int32_t split_count;  // entries taken in the split table
  int32_t help_cursor;  // entries below it are drained
  int32_t max_dplus;    // largest out-degree (bounds every w(u) by d+(u) max_dplus)
  int32_t pad[3];
};

// Equal-work quanta.  The work of a source is w(u) = sum of d+(v) over its
// middles v, the wedges it enumerates; a source whose out-list is searched in
// memory (d+(u) above kGlobalMin) counts each wedge kGlobalWeight times, for the
// binary search it costs.  A workgroup-mode source with such work above the
// quantum is cut into P = ceil(work / quantum) parts (at most kMaxParts):
// part k takes the middles k, k + P, k + 2P, ... (each part then holds about
// w(u) / P wedges).  Its workgroup publishes it in the split table, and parts
// are claimed through the entry's counter, by that workgroup and by any other
// that has run out of sources, so a heavy source no longer sets the tail.
constexpr int kSplitCap = 4096;       // split table entries (a fuller table keeps parts local)
constexpr int32_t kMaxParts = 1024;
constexpr int kSplitDefaultLog2 = 21;  // default quantum: 2^21 wedges
constexpr uint64_t kGlobalWeight = 8;

// The workgroup's schedule in LDS (written by thread 0).
constexpr int kSchedState = 0, kSchedU = 1, kSchedPart = 2, kSchedParts = 3, kSchedIdx = 4,
              kSchedEnt = 5, kSchedLocalK = 6, kSchedMaxD = 7, kSchedWords = 8;
constexpr int kHelpWindows = 4;  // 64-entry windows of the split table one step looks at
constexpr int32_t kStateDone = 0, kStateWork = 1, kStateNew = 2, kStateSkip = 3;
constexpr int32_t kNoEntry = -1, kLocalEntry = -2;

struct SplitEntry {
  unsigned long long word;  // (P << 32) | u once published, 0 before
  int32_t next;             // parts claimed so far
  int32_t pad;
};

constexpr int kSmallGrab = 16;  // wave-mode sources per run in the dynamic hand-out
static_assert(kSmallGrab <= kWave, "a run's sources are prefetched one per lane");

constexpr int kBinItems = 16;

// Out-degree of vertex base + r * 256 + tid for r < kBinItems, all loads in
// flight together (indices clamped to n - 1, n >= 1); -1 past n.
template <typename OffT>
__device__ __forceinline__ void bin_degrees(int64_t n, const OffT* __restrict__ row_ptr,
                                            int64_t base, int64_t (&d)[kBinItems]) {
  int64_t lo[kBinItems], hi[kBinItems];
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    const int64_t u = base + r * 256 + threadIdx.x;
    const int64_t c = u < n ? u : n - 1;
    lo[r] = row_ptr[c];
    hi[r] = row_ptr[c + 1];
  }
#pragma unroll
  for (int r = 0; r < kBinItems; ++r)
    d[r] = base + r * 256 + threadIdx.x < n ? hi[r] - lo[r] : -1;
}

// Sources per class: one workgroup per 256 * kBinItems vertices, one global
// atomic per class and workgroup.
template <typename OffT>
__global__ __launch_bounds__(256) void bin_count_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                        CountState* __restrict__ st, int small_max) {
  __shared__ int32_t h[kNumClasses + 1];
  if (threadIdx.x <= kNumClasses) h[threadIdx.x] = 0;
  __syncthreads();
  int64_t d[kBinItems];
  bin_degrees(n, row_ptr, (int64_t)blockIdx.x * (256 * kBinItems), d);
  int32_t mine[kNumClasses] = {0, 0, 0, 0, 0, 0, 0, 0};
  int32_t dmax = 0;
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    const int c = d[r] >= 0 ? source_class(d[r], small_max) : -1;
#pragma unroll
    for (int k = 0; k < kNumClasses; ++k) mine[k] += (c == k);
    dmax = d[r] > dmax ? (int32_t)d[r] : dmax;
  }
#pragma unroll
  for (int k = 0; k < kNumClasses; ++k) {
    const int64_t s = wave_sum(mine[k]);
    if (lane_id() == 0 && s) atomicAdd(&h[k], (int32_t)s);
  }
  dmax = read_lane(wave_inclusive_max32(dmax), kWave - 1);
  if (lane_id() == 0 && dmax) atomicMax(&h[kNumClasses], dmax);
  __syncthreads();
  if (threadIdx.x < kNumClasses && h[threadIdx.x]) atomicAdd(&st->class_count[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == kNumClasses && h[kNumClasses]) atomicMax(&st->max_dplus, h[kNumClasses]);
}

template <typename OffT>
__global__ __launch_bounds__(256) void bin_write_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                        CountState* __restrict__ st,
                                                        int32_t* __restrict__ list, int small_max) {
  __shared__ int32_t lcnt[kNumClasses];
  __shared__ int32_t gbase[kNumClasses];
  if (threadIdx.x < kNumClasses) lcnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * (256 * kBinItems);
  int64_t d[kBinItems];
  bin_degrees(n, row_ptr, base, d);
  int cls[kBinItems];
  int32_t lr[kBinItems];
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    cls[r] = d[r] >= 0 ? source_class(d[r], small_max) : -1;
    lr[r] = cls[r] >= 0 ? atomicAdd(&lcnt[cls[r]], 1) : 0;
  }
  __syncthreads();
  if (threadIdx.x < kNumClasses) {
    int32_t off = 0;
    for (int c = 0; c < (int)threadIdx.x; ++c) off += st->class_count[c];
    gbase[threadIdx.x] = off + (lcnt[threadIdx.x] ? atomicAdd(&st->class_cursor[threadIdx.x],
                                                              lcnt[threadIdx.x])
                                                  : 0);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    if (cls[r] >= 0) list[gbase[cls[r]] + lr[r]] = (int32_t)(base + r * 256 + threadIdx.x);
  }
}

// The source lists by class (n >= 1): counts, then the lists.
template <typename OffT>
void launch_bins(int64_t n, const OffT* row_ptr, CountState* st, int32_t* list, int small_max,
                 hipStream_t s) {
  const unsigned grid = (unsigned)((n + 256 * kBinItems - 1) / (256 * kBinItems));
  bin_count_kernel<OffT><<<grid, 256, 0, s>>>(n, row_ptr, st, small_max);
  bin_write_kernel<OffT><<<grid, 256, 0, s>>>(n, row_ptr, st, list, small_max);
}

__global__ void init_state_kernel(CountState* st, SplitEntry* split, uint64_t* total) {
  int32_t* p = reinterpret_cast<int32_t*>(st);
  for (int i = threadIdx.x; i < (int)(sizeof(CountState) / 4); i += blockDim.x) p[i] = 0;
  int32_t* q = reinterpret_cast<int32_t*>(split);
  for (int i = threadIdx.x; i < kSplitCap * (int)(sizeof(SplitEntry) / 4); i += blockDim.x) q[i] = 0;
  if (threadIdx.x == 0) *total = 0;
}

__global__ void zero_u64_kernel(uint64_t* p, int64_t len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0;
}

// One LDS cuckoo table (plus its stash).  In the sorted mode slot[0, keys)
// holds the keys in ascending order instead.
struct Table {
  int32_t* slot;       // [2 * side]; halves [0, side) and [side, 2 * side)
  uint32_t* cnt;       // [2 * side] hit counters (per-vertex mode only)
  int32_t* stash;      // [kStash]
  uint32_t* stash_cnt; // [kStash]
  int32_t* meta;       // [0] stash entries, [1] overflow flag, [2] broadcast slot
};

template <bool PV>
__device__ __forceinline__ Table table_at(char* base, int side_max) {
  Table t;
  t.slot = reinterpret_cast<int32_t*>(base);
  char* p = base + 2 * side_max * 4;
  t.cnt = reinterpret_cast<uint32_t*>(p);
  if (PV) p += 2 * side_max * 4;
  t.stash = reinterpret_cast<int32_t*>(p);
  p += kStash * 4;
  t.stash_cnt = reinterpret_cast<uint32_t*>(p);
  p += kStash * 4;
  t.meta = reinterpret_cast<int32_t*>(p);
  return t;
}

// Group = one wave (Waves == 1) or the whole workgroup (Waves == kWavesPerBlock).
template <int Waves>
__device__ __forceinline__ void group_sync() {
  if (Waves == 1) wave_sync();
  else __syncthreads();
}

template <int Waves>
__device__ __forceinline__ int group_rank() {
  return Waves == 1 ? lane_id() : (int)threadIdx.x;
}

// log2 of the slots per half for `keys` keys: load <= 0.4 over both halves.
__host__ __device__ constexpr int side_log2(int keys) {
  const int want = keys + (keys >> 2) + 1;
  int b = 4;
  while ((1 << b) < want) ++b;
  return b;
}
static_assert((1 << side_log2(kSmallMax)) <= kSmallSide, "wave-mode table too small");
static_assert((1 << side_log2(kChunk)) <= kSideMax, "workgroup-mode table too small");

struct Slice {
  int side;   // slots per cuckoo half
  int shift;  // 32 - log2(side)
  int keys;   // keys in this slice
  int stash_n;
  const int32_t* gkeys;  // kModeGlobal: the sorted row N+(u) in memory
};

// Binary search of the sorted slice (the fallback mode): whether w is a key.
template <bool PV>
__device__ __forceinline__ bool probe_sorted(const Table& t, const Slice& sl, int32_t w) {
  int lo = 0, len = sl.keys;
  while (len > 0) {
    const int half = len >> 1;
    if (t.slot[lo + half] < w) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  const bool hit = lo < sl.keys && t.slot[lo] == w;
  if (PV && hit) atomicAdd(&t.cnt[lo], 1u);
  return hit;
}

// The wave's hits as a mask, counting each hit on its slot (per-slot counter
// kinds) and, with Seg, on the caller's per-lane LDS counter `seg` too.  The two
// slot compares are balloted directly and the same compare results select the
// lanes that add to the counters, so no per-lane boolean is rebuilt from the
// mask.
template <int Mode, bool Wide, bool Seg>
__device__ __forceinline__ uint64_t probe_counted(const Table& t, const Slice& sl, int32_t w,
                                                  uint32_t* seg) {
  if (Mode == kModeSorted) {
    const bool h = probe_sorted<true>(t, sl, w);
    if (Seg && h) atomicAdd(seg, 1u);
    return ballot(h);
  }
  // byte offsets of the two slots, shared by the key and the counter arrays
  const uint32_t p = hash_product(hash_input<Wide>(w));
  const uint32_t oa = slot_a_of(p, sl.shift) * 4u;
  const uint32_t ob = (uint32_t)sl.side * 4u + slot_b_of(p, sl.shift) * 4u;
  const int32_t a = *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(t.slot) + oa);
  const int32_t b = *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(t.slot) + ob);
  const bool ha = a == w;
  const bool hb = b == w;
  uint64_t m = ballot(ha) | ballot(hb);
  if (ha | hb) {
    atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(t.cnt) + (ha ? oa : ob)), 1u);
    if (Seg) atomicAdd(seg, 1u);
  }
  if (Mode == kModeStash) {
    for (int i = 0; i < sl.stash_n; ++i) {
      const bool h = t.stash[i] == w;
      m |= ballot(h);
      if (h) {
        atomicAdd(&t.stash_cnt[i], 1u);
        if (Seg) atomicAdd(seg, 1u);
      }
    }
  }
  return m;
}

// The wave's hits as a mask.  Without per-slot counters the two slot compares
// are balloted directly (no per-lane boolean is materialised).
template <bool PV, int Mode, bool Wide>
__device__ __forceinline__ uint64_t probe_ballot(const Table& t, const Slice& sl, int32_t w) {
  if (PV) return probe_counted<Mode, Wide, false>(t, sl, w, nullptr);
  if (Mode == kModeSorted) return ballot(probe_sorted<false>(t, sl, w));
  const uint32_t p = hash_product(hash_input<Wide>(w));
  const int32_t a = t.slot[slot_a_of(p, sl.shift)];
  const int32_t b = t.slot[(uint32_t)sl.side + slot_b_of(p, sl.shift)];
  uint64_t m = ballot(a == w) | ballot(b == w);
  if (Mode == kModeStash) {
    for (int i = 0; i < sl.stash_n; ++i) m |= ballot(t.stash[i] == w);
  }
  return m;
}

// Element i of a list by a 32-bit unsigned byte offset from its (uniform) start,
// which lets the load take the scalar-base + vector-offset form.
__device__ __forceinline__ int32_t list_at(const int32_t* __restrict__ lst, uint32_t i) {
  return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(lst) + i * 4u);
}

// Listing output of one source u: its rows start at `base`; a group-shared LDS
// cursor hands out row slots as hits arrive (rows of one source are
// contiguous, in no particular order).
// Support mode reuses it for the edge counters: sup[e] for e an index into the
// column array, and ubeg = the first edge of u.
struct ListCtx {
  int32_t* out;     // int32[3 * cap]
  int64_t base;
  int64_t cap;
  int32_t* cursor;  // LDS
  int32_t u;
  uint32_t* sup;
  int64_t ubeg;
  uint64_t* tv;  // per-vertex counts (kModeGlobal adds t(w) per hit)
  const uint8_t* dir;   // directed kind: a 2-bit code per DAG edge (arc directions or label)
  const uint32_t* tab;  // directed kind: matches per triangle by its three codes (LDS)
};

// Writes the wedges u -> v -> w of the lanes set in `hits` as rows (u, v, w).
// Called by the whole wave (lane 0 takes the slots).
__device__ __forceinline__ void emit(const ListCtx& c, uint64_t hits, int32_t v, int32_t w) {
  if (!hits) return;
  int32_t start = 0;
  if (lane_id() == 0) start = atomicAdd(c.cursor, (int32_t)popc(hits));
  start = read_lane(start, 0);  // a scalar read, no LDS round trip
  if ((hits >> lane_id()) & 1u) {
    const int64_t row = c.base + start + rank_below(hits);
    if (row < c.cap) {
      int32_t* o = c.out + 3 * row;
      o[0] = c.u;
      o[1] = v;
      o[2] = w;
    }
  }
}

// Position of w in the sorted keys[0, n) in memory, or -1.
__device__ __forceinline__ int32_t find_sorted(const int32_t* __restrict__ keys, int32_t n,
                                               int32_t w) {
  int32_t lo = 0, len = n;
  while (len > 0) {
    const int32_t half = len >> 1;
    if (keys[lo + half] < w) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo < n && keys[lo] == w ? lo : -1;
}

// Directed kind: the code of the edge (u, w) when w is a key of the
// slice (stored beside the key when the table was built), else -1.
template <int Mode, bool Wide>
__device__ __forceinline__ int32_t probe_code(const Table& t, const Slice& sl, int32_t w,
                                              const ListCtx& lc) {
  if (Mode == kModeGlobal) {
    const int32_t pos = find_sorted(sl.gkeys, sl.keys, w);
    return pos >= 0 ? (int32_t)lc.dir[lc.ubeg + pos] : -1;
  }
  if (Mode == kModeSorted) {
    int lo = 0, len = sl.keys;
    while (len > 0) {
      const int half = len >> 1;
      if (t.slot[lo + half] < w) {
        lo += half + 1;
        len -= half + 1;
      } else {
        len = half;
      }
    }
    return lo < sl.keys && t.slot[lo] == w ? (int32_t)t.cnt[lo] : -1;
  }
  const uint32_t p = hash_product(hash_input<Wide>(w));
  const uint32_t sa = slot_a_of(p, sl.shift);
  const uint32_t sb = (uint32_t)sl.side + slot_b_of(p, sl.shift);
  if (t.slot[sa] == w) return (int32_t)t.cnt[sa];
  if (t.slot[sb] == w) return (int32_t)t.cnt[sb];
  if (Mode == kModeStash) {
    for (int i = 0; i < sl.stash_n; ++i)
      if (t.stash[i] == w) return (int32_t)t.stash_cnt[i];
  }
  return -1;
}

// The matches of a directed query on the triangle u -> v -> w: the table entry
// of its three direction codes, 16 c(u, v) + 4 c(u, w) + c(v, w); 0 on a miss.
// The code of (v, w) is loaded beside w itself (the same position of the column
// array), so no hit waits for a load after its probe.
__device__ __forceinline__ uint32_t directed_hits(const ListCtx& lc, uint32_t cuv16, int32_t cuw,
                                                  uint32_t cvw) {
  return cuw >= 0 ? lc.tab[cuv16 + 4u * (uint32_t)cuw + cvw] : 0u;
}

// The wave's hits among the wedges u -> v -> w[lane], with the per-hit work of
// each kind: LDS slot counters, or (kModeGlobal, which has no table) the
// per-vertex count t(w) and the support of (u, w) directly.  With Seg (counted
// kinds only) each hit also adds one to the lane's LDS counter `seg`.
template <int K, int Mode, bool Wide, bool Seg = false>
__device__ __forceinline__ uint64_t probe_mask(const Table& t, const Slice& sl, int32_t w,
                                               const ListCtx& lc, uint32_t* seg = nullptr) {
  if (Mode == kModeGlobal) {
    const int32_t pos = find_sorted(sl.gkeys, sl.keys, w);
    if (K == kKindPerVertex && pos >= 0)
      atomicAdd((unsigned long long*)&lc.tv[w], 1ull);
    if (K == kKindSupport && pos >= 0) atomicAdd(&lc.sup[lc.ubeg + pos], 1u);
    if (Seg && pos >= 0) atomicAdd(seg, 1u);
    return ballot(pos >= 0);
  }
  if (counted(K)) return probe_counted<Mode, Wide, Seg>(t, sl, w, seg);
  return probe_ballot<false, Mode, Wide>(t, sl, w);
}

// Hits among the `len` ids of one out-neighbour list `lst` (len >= 1).  Four
// 64-wide loads are issued before any probe so each wave keeps several memory
// requests in flight; the tail clamps its indices to stay inside the list.
template <int K, int Mode, bool Wide>
__device__ __forceinline__ uint32_t scan_list(const int32_t* __restrict__ lst, int len,
                                              const Table& t, const Slice& sl, int32_t v,
                                              const ListCtx& lc, int64_t jb, uint32_t cuv16) {
  const int lane = lane_id();
  uint32_t hv = 0;
  int base = 0;
  for (; base + kUnroll * kWave <= len; base += kUnroll * kWave) {
    const int32_t* p = lst + base + lane;
    int32_t w[kUnroll];
    uint32_t cw[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      w[k] = p[k * kWave];
      cw[k] = K == kKindDirected ? (uint32_t)lc.dir[jb + base + k * kWave + lane] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      if (K == kKindDirected) {
        hv += directed_hits(lc, cuv16, probe_code<Mode, Wide>(t, sl, w[k], lc), cw[k]);
        continue;
      }
      const uint64_t b = probe_mask<K, Mode, Wide>(t, sl, w[k], lc);
      hv += popc(b);
      if (K == kKindList) emit(lc, b, v, w[k]);
      if (K == kKindSupport && ((b >> lane) & 1u))
        atomicAdd(&lc.sup[jb + base + k * kWave + lane], 1u);  // the edge (v, w)
    }
  }
  if (base < len) {
    const uint32_t last = (uint32_t)(len - 1);
    int32_t w[kUnroll];
    uint32_t cw[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint32_t i = (uint32_t)(base + k * kWave + lane);
      const int32_t x = list_at(lst, i < last ? i : last);
      w[k] = i <= last ? x : kNoKey;
      cw[k] = K == kKindDirected ? (uint32_t)lc.dir[jb + (i < last ? i : last)] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      if (base + k * kWave < len) {
        if (K == kKindDirected) {
          hv += directed_hits(lc, cuv16, probe_code<Mode, Wide>(t, sl, w[k], lc), cw[k]);
          continue;
        }
        const uint64_t b = probe_mask<K, Mode, Wide>(t, sl, w[k], lc);
        hv += popc(b);
        if (K == kKindList) emit(lc, b, v, w[k]);
        if (K == kKindSupport && ((b >> lane) & 1u))
          atomicAdd(&lc.sup[jb + base + k * kWave + lane], 1u);  // the edge (v, w)
      }
    }
  }
  return hv;
}

// Adds c to the per-slot counter of key v (counted kinds), for a v that is in
// the table: a middle of the source, when the table holds all of N+(u).  The
// (u, v) counts then reach memory with the slot's own flush at the end of the
// source instead of one global atomic per middle; such an atomic, although
// nothing waits for its value, holds up the wave's next wait on a list load.
template <int Mode, bool Wide>
__device__ __forceinline__ void slot_add(const Table& t, const Slice& sl, int32_t v, uint32_t c) {
  if (Mode == kModeSorted) {
    int lo = 0, len = sl.keys;
    while (len > 0) {
      const int half = len >> 1;
      if (t.slot[lo + half] < v) {
        lo += half + 1;
        len -= half + 1;
      } else {
        len = half;
      }
    }
    atomicAdd(&t.cnt[lo], c);
    return;
  }
  const uint32_t p = hash_product(hash_input<Wide>(v));
  const uint32_t s1 = slot_a_of(p, sl.shift);
  if (t.slot[s1] == v) {
    atomicAdd(&t.cnt[s1], c);
    return;
  }
  const uint32_t s2 = (uint32_t)sl.side + slot_b_of(p, sl.shift);
  if (t.slot[s2] == v) {
    atomicAdd(&t.cnt[s2], c);
    return;
  }
  if (Mode == kModeStash) {
    for (int i = 0; i < sl.stash_n; ++i) {
      if (t.stash[i] == v) {
        atomicAdd(&t.stash_cnt[i], c);
        return;
      }
    }
  }
}

// The short out-lists of up to 64 middles held one per lane (len = 0 for lanes
// without one) walked as one concatenation, kWin * 64 wedges per step, so a
// wave is not spent on a single short list.  Lane l's segment is the last lane
// whose list starts at or before its position: each list's first position is
// marked in LDS and propagated with a wave max-scan.  The marker array holds -1
// between walks (the writer clears its own entry after the step; a wave's LDS
// operations complete in program order).  Returns the hits (uniform); counted
// kinds also get each lane's own list's hits in *seg_hits.
template <int K, int Mode, bool Wide, typename OffT>
__device__ __forceinline__ uint32_t scan_short(int32_t v, OffT vb, int32_t len,
                                               const int32_t* __restrict__ col, const Table& t,
                                               const Slice& sl, const WaveScratch& ws,
                                               const ListCtx& lc, uint32_t* seg_hits,
                                               uint32_t cuv16) {
  constexpr bool CNT = counted(K);
  const int lane = lane_id();
  const int32_t incl = wave_inclusive_sum32(len);
  const int32_t start = incl - len;
  const int32_t total = read_lane(incl, kWave - 1);
  // walk position pos of this lane's list is col[pos + delta]
  const OffT delta = vb - (OffT)start;
  if (CNT) ws.shits[lane] = 0;
  int32_t carry = -1;
  uint32_t hv = 0;
  for (int32_t base = 0; base < total; base += kWin * kWave) {
    const bool marks = len > 0 && start >= base && start < base + kWin * kWave;
    if (marks) ws.mark[start - base] = lane;
    wave_sync();
    int32_t seg[kWin];
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      int32_t sk = wave_inclusive_max32(ws.mark[k * kWave + lane]);
      sk = sk > carry ? sk : carry;
      carry = read_lane(sk, kWave - 1);
      seg[k] = sk;
    }
    wave_sync();
    if (marks) ws.mark[start - base] = -1;
    int32_t w[kWin], mid[kWin];
    uint32_t c16[kWin], cvw[kWin];
    OffT at[kWin];  // column index; int32 offsets keep the address arithmetic 32-bit
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      const int32_t pos = base + k * kWave + lane;
      const int32_t sk = seg[k] < 0 ? 0 : seg[k];
      mid[k] = K == kKindList ? __shfl(v, sk, kWave) : 0;
      c16[k] = K == kKindDirected ? (uint32_t)__shfl((int32_t)cuv16, sk, kWave) : 0u;
      // the segment's list is the last non-empty one starting at or before pos,
      // so for pos < total, start(sk) <= pos < start(sk) + len(sk)
      at[k] = (OffT)pos + __shfl(delta, sk, kWave);
      if (sizeof(OffT) == 4)
        w[k] = pos < total ? list_at(col, (uint32_t)at[k]) : kNoKey;
      else
        w[k] = pos < total ? col[at[k]] : kNoKey;
      cvw[k] = K == kKindDirected && pos < total ? (uint32_t)lc.dir[at[k]] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      if (base + k * kWave < total) {
        if (K == kKindDirected) {
          hv += directed_hits(lc, c16[k], probe_code<Mode, Wide>(t, sl, w[k], lc), cvw[k]);
          continue;
        }
        // a hit adds to its segment's counter inside the probe (counted kinds)
        const uint64_t b = probe_mask<K, Mode, Wide, CNT>(t, sl, w[k], lc,
                                                          &ws.shits[seg[k] < 0 ? 0 : seg[k]]);
        if (K == kKindSupport && ((b >> lane) & 1u))
          atomicAdd(&lc.sup[at[k]], 1u);  // the edge (v, w)
        hv += popc(b);
        if (K == kKindList) emit(lc, b, mid[k], w[k]);
      }
    }
  }
  if (CNT) {
    wave_sync();
    *seg_hits = ws.shits[lane];
  }
  return hv;
}

// One of the equal-work parts of a split source: the middles i = part + j parts.
struct Part {
  int64_t part;
  int64_t parts;
};

// All middles v of source u handled by this wave: v = N+(u)[i] for
// i = gwave, gwave + Waves, ...; 64 of them are prefetched per batch.  Lists of
// kShortMax or more ids are streamed one at a time; shorter ones are walked
// together by scan_short.  Empty lists add nothing (1-look-ahead).
template <int Waves, int K, int Mode, bool Wide, typename OffT>
__device__ uint64_t scan_middles(const int32_t* __restrict__ nbrs, int64_t d,
                                 const OffT* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                 uint64_t* __restrict__ tv, const Table& t, const Slice& sl,
                                 const WaveScratch& ws, const ListCtx& lc, const Part& pt) {
  constexpr bool PV = K == kKindPerVertex;
  const int lane = lane_id();
  const int gwave = Waves == 1 ? 0 : (int)threadIdx.x / kWave;
  // every middle is a key of this table (one slice): (u, v) counts go to its slot
  const bool local_v = Mode != kModeGlobal && (int64_t)sl.keys == d;
  // a workgroup-mode source may be split: part k of P takes the middles i = k + j P
  const int64_t first = Waves > 1 ? pt.part : 0;
  const int64_t stride = Waves > 1 ? pt.parts : 1;
  const int64_t mine = first < d ? (d - first + stride - 1) / stride : 0;
  uint64_t src_hits = 0;
  for (int64_t i0 = 0; i0 < mine; i0 += (int64_t)Waves * kWave) {
    const int64_t j = i0 + (int64_t)Waves * lane + gwave;
    const int64_t i = first + j * stride;
    int32_t v = 0;
    OffT vb = 0, ve = 0;
    uint32_t cuv16 = 0;  // directed kind: 16 x the code of (u, v)
    if (j < mine) {
      v = nbrs[i];
      vb = row_ptr[v];
      ve = row_ptr[v + 1];
      if (K == kKindDirected) cuv16 = 16u * lc.dir[lc.ubeg + i];
    }
    const int64_t len = (int64_t)(ve - vb);
    // Only the main probe mode walks short lists together (keeps the rare modes small).
    const uint64_t shorts = Mode == kModeCuckoo ? ballot(len > 0 && len < kShortMax) : 0;
    const bool walk_short = popc(shorts) >= kShortMinLists;
    uint64_t longs = walk_short ? ballot(len >= kShortMax) : ballot(len > 0);
    uint32_t cv = 0;  // counted kinds: the (u, v) hits of this lane's middle
    while (longs) {
      const int j = __builtin_ctzll(longs);
      longs &= longs - 1;
      int64_t jb, je;
      if (sizeof(OffT) == 4) {
        jb = read_lane((int32_t)vb, j);
        je = read_lane((int32_t)ve, j);
      } else {
        jb = read_lane64((int64_t)vb, j);
        je = read_lane64((int64_t)ve, j);
      }
      const int32_t vj = read_lane(v, j);
      const uint32_t cj = K == kKindDirected ? (uint32_t)read_lane((int32_t)cuv16, j) : 0u;
      const uint32_t hv = scan_list<K, Mode, Wide>(col + jb, (int)(je - jb), t, sl, vj, lc, jb, cj);
      src_hits += hv;
      if (counted(K) && lane == j) cv = hv;
    }
    if (walk_short) {
      const bool is_short = len > 0 && len < kShortMax;
      uint32_t cs = 0;
      src_hits += scan_short<K, Mode, Wide, OffT>(v, vb, is_short ? (int32_t)len : 0, col, t, sl,
                                                  ws, lc, &cs, cuv16);
      cv += cs;
    }
    // the (u, v) counts of the batch's middles, all lanes at once
    if (counted(K) && cv) {
      if (local_v) {
        slot_add<Mode, Wide>(t, sl, v, cv);  // t(v), or the edge (u, v)
      } else {
        if (PV) atomicAdd((unsigned long long*)&tv[v], (unsigned long long)cv);
        if (K == kKindSupport) atomicAdd(&lc.sup[lc.ubeg + i], cv);  // the edge (u, v)
      }
    }
  }
  return src_hits;
}

// Where the listing pass writes (rows of source u start at off[u]), and the
// edge counters of the support pass.
struct ListArgs {
  int32_t* out;
  const int64_t* off;
  int64_t cap;
  uint32_t* sup;
  const uint8_t* dir;   // directed kind: a 2-bit code per DAG edge
  const uint32_t* tab;  // directed kind: set by the kernel (its LDS copy of the table)
};

// Count of key w in the slice's table (the per-slot counters).
template <bool Wide>
__device__ __forceinline__ uint32_t slot_count(const Table& t, const Slice& sl, int mode,
                                               int p, int32_t w) {
  if (mode == kModeSorted) return t.cnt[p];
  const uint32_t hp = hash_product(hash_input<Wide>(w));
  const uint32_t s1 = slot_a_of(hp, sl.shift);
  const uint32_t s2 = (uint32_t)sl.side + slot_b_of(hp, sl.shift);
  if (t.slot[s1] == w) return t.cnt[s1];
  if (t.slot[s2] == w) return t.cnt[s2];
  for (int i = 0; i < sl.stash_n; ++i)
    if (t.stash[i] == w) return t.stash_cnt[i];
  return 0;
}

// Process one source u (its out-list at col[beg, beg + d)) with a group of
// Waves waves sharing table `t`.  Returns this wave's hit count (uniform across
// the wave).

template <int Waves, int K, bool Wide, typename OffT>
__device__ uint64_t process_source(int64_t u, int64_t beg, int64_t d,
                                   const OffT* __restrict__ row_ptr,
                                   const int32_t* __restrict__ col, uint64_t* __restrict__ tv,
                                   const Table& t, const WaveScratch& ws, int max_keys,
                                   int max_kicks, bool force_sorted, const ListArgs& la,
                                   const Part& pt) {
  constexpr bool PV = K == kKindPerVertex;
  constexpr bool CNT = counted(K);
  const int lane = lane_id();
  const int gr = group_rank<Waves>();
  const int32_t* nbrs = col + beg;
  uint64_t wave_hits = 0;
  ListCtx lc{la.out, 0, la.cap, t.meta + 3, (int32_t)u, la.sup, beg, tv, la.dir, la.tab};
  if (K == kKindList) {
    lc.base = la.off[u];
    if (gr == 0) t.meta[3] = 0;  // ordered before any hit by the next barrier
  }
  if (Waves > 1 && d > kGlobalMin) {
    // Too many slices: every slice would stream all of the N+(v) again.  Binary
    // search the sorted row in memory instead (no table, counts added per hit).
    if (K == kKindList) group_sync<Waves>();
    Slice sl;
    sl.keys = (int)d;
    sl.side = 0;
    sl.shift = 0;
    sl.stash_n = 0;
    sl.gkeys = nbrs;
    const uint64_t src_hits =
        scan_middles<Waves, K, kModeGlobal, Wide, OffT>(nbrs, d, row_ptr, col, tv, t, sl, ws, lc, pt);
    if (PV && src_hits && lane == 0)
      atomicAdd((unsigned long long*)&tv[u], (unsigned long long)src_hits);
    group_sync<Waves>();
    return src_hits;
  }
  for (int64_t c0 = 0; c0 < d; c0 += max_keys) {
    Slice sl;
    sl.keys = (int)(d - c0 < max_keys ? d - c0 : max_keys);
    const int b = side_log2(sl.keys);
    sl.side = 1 << b;
    sl.shift = 32 - b;
    for (int s = gr; s < 2 * sl.side; s += Waves * kWave) {
      t.slot[s] = kEmpty;
      if (CNT) t.cnt[s] = 0;
    }
    if (gr < kStash) t.stash_cnt[gr] = 0;
    if (gr < 2) t.meta[gr] = 0;
    group_sync<Waves>();
    for (int i = gr; i < sl.keys; i += Waves * kWave) {
      int32_t cur = nbrs[c0 + i];
      int hs = 0;
      for (int kick = 0; kick < max_kicks && cur != kEmpty; ++kick) {
        const uint32_t s = hs ? (uint32_t)sl.side + hash_b<Wide>(cur, sl.shift)
                              : hash_a<Wide>(cur, sl.shift);
        cur = atomicExch(&t.slot[s], cur);
        hs ^= 1;
      }
      if (cur != kEmpty) {
        const int at = atomicAdd(&t.meta[0], 1);
        if (at < kStash) t.stash[at] = cur;
        else t.meta[1] = 1;
      }
    }
    group_sync<Waves>();
    const int stash_raw = t.meta[0];
    sl.stash_n = stash_raw < kStash ? stash_raw : kStash;
    const int mode =
        (force_sorted || t.meta[1]) ? kModeSorted : (sl.stash_n ? kModeStash : kModeCuckoo);
    if (mode == kModeSorted) {
      // N+(u) rows are sorted: copy the slice into the slot array for binary search
      group_sync<Waves>();
      for (int i = gr; i < sl.keys; i += Waves * kWave) t.slot[i] = nbrs[c0 + i];
      group_sync<Waves>();
    }
    if (K == kKindDirected) {
      // the direction code of (u, key) beside every key of the slice
      for (int p = gr; p < sl.keys; p += Waves * kWave) {
        const uint32_t code = la.dir[beg + c0 + p];
        if (mode == kModeSorted) {
          t.cnt[p] = code;  // slot p holds the slice's p-th key
          continue;
        }
        const int32_t w = nbrs[c0 + p];
        const uint32_t hp = hash_product(hash_input<Wide>(w));
        const uint32_t s1 = slot_a_of(hp, sl.shift);
        const uint32_t s2 = (uint32_t)sl.side + slot_b_of(hp, sl.shift);
        if (t.slot[s1] == w) {
          t.cnt[s1] = code;
        } else if (t.slot[s2] == w) {
          t.cnt[s2] = code;
        } else {
          for (int i = 0; i < sl.stash_n; ++i)
            if (t.stash[i] == w) t.stash_cnt[i] = code;
        }
      }
      group_sync<Waves>();
    }
    uint64_t src_hits;
    if (mode == kModeCuckoo)
      src_hits = scan_middles<Waves, K, kModeCuckoo, Wide, OffT>(nbrs, d, row_ptr, col, tv, t, sl, ws, lc, pt);
    else if (mode == kModeStash)
      src_hits = scan_middles<Waves, K, kModeStash, Wide, OffT>(nbrs, d, row_ptr, col, tv, t, sl, ws, lc, pt);
    else
      src_hits = scan_middles<Waves, K, kModeSorted, Wide, OffT>(nbrs, d, row_ptr, col, tv, t, sl, ws, lc, pt);
    wave_hits += src_hits;
    if (K == kKindSupport) {
      // the edges (u, w): hits counted on w's slot
      group_sync<Waves>();
      for (int p = gr; p < sl.keys; p += Waves * kWave) {
        const uint32_t c = slot_count<Wide>(t, sl, mode, p, nbrs[c0 + p]);
        if (c) atomicAdd(&la.sup[beg + c0 + p], c);
      }
    }
    if (PV) {
      if (src_hits && lane == 0) atomicAdd((unsigned long long*)&tv[u], (unsigned long long)src_hits);
      group_sync<Waves>();
      if (mode == kModeSorted) {
        for (int p = gr; p < sl.keys; p += Waves * kWave) {
          const uint32_t c = t.cnt[p];
          if (c) atomicAdd((unsigned long long*)&tv[t.slot[p]], (unsigned long long)c);
        }
      } else {
        for (int s = gr; s < 2 * sl.side; s += Waves * kWave) {
          const int32_t k = t.slot[s];
          const uint32_t c = t.cnt[s];
          if (k != kEmpty && c) atomicAdd((unsigned long long*)&tv[k], (unsigned long long)c);
        }
        if (gr < sl.stash_n && t.stash_cnt[gr])
          atomicAdd((unsigned long long*)&tv[t.stash[gr]], (unsigned long long)t.stash_cnt[gr]);
      }
    }
    group_sync<Waves>();
  }
  return wave_hits;
}

// Runtime parameters of one count launch.
// Matches of a directed query on one triangle u -> v -> w of the DAG, by the
// direction codes of its edges: entry 16 c(u, v) + 4 c(u, w) + c(v, w).
struct DirCodes {
  uint8_t v[64];
};

struct CountArgs {
  SplitEntry* split;   // split table (kSplitCap entries)
  int32_t split_shift;  // log2 of the wedges per part of a split source; 0: never split
  const int32_t* gid;  // batched mode: graph of each vertex (-1: none); else null
  uint64_t* totals;    // batched mode: per-graph totals; else null
  uint64_t* src_cnt;   // listing, first pass: hits of each source; else null
  const int64_t* list_status;  // listing pass: the row count, negative if over capacity
  ListArgs list;
  int max_kicks;
  int force_sorted;
  DirCodes codes;  // directed kind only
};

// Persistent count kernel: workgroup-mode sources first (largest class first,
// through a global cursor after a static first round), then wave-mode sources
// round robin.  In batched mode each source's hits are also added to the total
// of its graph.
template <int K, bool Wide, typename OffT>
__global__ __launch_bounds__(kBlock, 8) void count_kernel(const OffT* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ list,
                                                       CountState* __restrict__ st,
                                                       uint64_t* __restrict__ total,
                                                       uint64_t* __restrict__ tv, CountArgs args) {
  constexpr bool PV = slot_words(K);  // table layout with a word per slot
  __shared__ __align__(16) char smem[smem_total(PV)];
  __shared__ uint32_t dtab[K == kKindDirected ? 64 : 1];
  if ((K == kKindList || K == kKindSupport) && *args.list_status < 0) return;
  ListArgs la = args.list;
  if (K == kKindDirected) {
    if (threadIdx.x < 64) dtab[threadIdx.x] = args.codes.v[threadIdx.x];
    __syncthreads();
    la.tab = dtab;
  }
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  WaveScratch ws;
  {
    char* p = smem + smem_bytes(PV) + wave * seg_bytes_per_wave(PV);
    ws.mark = reinterpret_cast<int32_t*>(p);
    ws.shits = reinterpret_cast<uint32_t*>(p + kWin * kWave * 4);
#pragma unroll
    for (int k = 0; k < kWin; ++k) ws.mark[k * kWave + lane] = -1;
    wave_sync();
  }
  int32_t n_large = 0;
  for (int c = 0; c < kNumClasses - 1; ++c) n_large += st->class_count[c];
  const int32_t n_small = st->class_count[kNumClasses - 1];
  uint64_t hits = 0;
  // Batched mode: this wave's hits of the graph it is working on, added to the
  // graph's total when the wave moves to another graph (consecutive sources are
  // mostly of one graph; one atomic per source would pile up on a few totals).
  int32_t pend_g = -1;
  uint64_t pend_h = 0;
  auto credit = [&](int32_t u, uint64_t h) {
    if (!args.totals || !h) return;
    const int32_t g = args.gid[u];
    if (g != pend_g) {
      if (pend_h && lane == 0) atomicAdd((unsigned long long*)&args.totals[pend_g], (unsigned long long)pend_h);
      pend_g = g;
      pend_h = 0;
    }
    if (g >= 0) pend_h += h;
  };

  // Workgroup-mode sources.  Thread 0 schedules, the workgroup follows: the
  // next piece of work is a part of the split source being drained, else the
  // next source of the list (its first one static, by the workgroup's id, later
  // ones from the cursor), else, once the list is used up, a part of a split
  // source some other workgroup published.  The schedule lives in LDS so that
  // process_source has one call site.
  const Table big = table_at<PV>(smem, kSideMax);
  __shared__ int32_t sched[kSchedWords];
  const bool splitting = K != kKindList && args.split_shift != 0;
  if (threadIdx.x == 0) {
    sched[kSchedIdx] = blockIdx.x;
    sched[kSchedEnt] = kNoEntry;
    // read once per workgroup: the state's cache line takes the cursor atomics
    sched[kSchedMaxD] = st->max_dplus;
  }
  while (true) {
    __syncthreads();  // every thread has read the previous step's schedule
    if (wave == 0) {
      if (lane == 0) {
        int32_t state = kStateDone;
        int32_t ent = sched[kSchedEnt];
        if (ent != kNoEntry) {
          const int32_t k = ent >= 0 ? atomicAdd(&args.split[ent].next, 1) : sched[kSchedLocalK]++;
          if (k < sched[kSchedParts]) {
            sched[kSchedPart] = k;
            state = kStateWork;
          } else {
            ent = kNoEntry;
          }
        }
        if (state == kStateDone && sched[kSchedIdx] < n_large) {
          sched[kSchedU] = list[sched[kSchedIdx]];
          sched[kSchedIdx] = (int32_t)gridDim.x + atomicAdd(&st->large_cursor, 1);
          state = kStateNew;
        }
        sched[kSchedEnt] = ent;
        sched[kSchedState] = state;
      }
      wave_sync();
      if (sched[kSchedState] == kStateDone && splitting) {
        // Out of sources: look for an open part in a few 64-entry windows of the
        // split table from the shared cursor (entries below it are drained).  An
        // unpublished entry reads 0 and is left to the workgroup that reserved
        // it, which claims every part nobody else takes.
        int32_t end = 0, at = 0;
        if (lane == 0) {
          end = __hip_atomic_load(&st->split_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          at = __hip_atomic_load(&st->help_cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        end = read_lane(end, 0);
        end = end < kSplitCap ? end : kSplitCap;
        at = read_lane(at, 0);
        for (int win = 0; win < kHelpWindows && at < end; ++win) {
          const int32_t e = at + lane;
          unsigned long long word = 0;
          int32_t nx = 0;
          if (e < end) {
            word = __hip_atomic_load(&args.split[e].word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            nx = __hip_atomic_load(&args.split[e].next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          const int32_t parts = (int32_t)(word >> 32);
          const uint64_t open = ballot(word != 0 && nx < parts);
          const uint64_t drained = ballot(word != 0 && nx >= parts);
          // entries drained in a row from the window's start: nobody needs them again
          const int lead = (int)__builtin_ctzll(~drained);
          if (lane == 0 && lead > 0) atomicMax(&st->help_cursor, at + lead);
          if (open) {
            const int j = (int)__builtin_ctzll(open);
            int32_t got = 0;
            if (lane == j) {
              const int32_t k = atomicAdd(&args.split[e].next, 1);
              if (k < parts) {
                sched[kSchedEnt] = e;
                sched[kSchedU] = (int32_t)(uint32_t)word;
                sched[kSchedParts] = parts;
                sched[kSchedPart] = k;
                sched[kSchedState] = kStateWork;
                got = 1;
              }
            }
            if (read_lane(got, j)) break;
            continue;  // lost the race for that entry: look at the same window again
          }
          at += kWave;
        }
      }
    }
    __syncthreads();
    const int32_t state = sched[kSchedState];
    if (state == kStateDone) break;
    const int32_t u = sched[kSchedU];
    const int64_t beg = row_ptr[u];
    const int64_t d = (int64_t)row_ptr[u + 1] - beg;
    if (state == kStateNew) {
      // a new source: its work w(u), the out-degrees of its middles summed over
      // the workgroup, decides whether it is split
      int32_t parts = 1;
      const uint64_t weight = d > kGlobalMin ? kGlobalWeight : 1;
      // w(u) <= d+(u) max_dplus: compute it only when that bound reaches the quantum
      // (compared in float, no 64-bit division; a loose bound only costs a sum)
      if (splitting && (float)d * (float)sched[kSchedMaxD] * (float)weight >=
                           (float)(uint64_t(1) << args.split_shift)) {
        uint64_t w = 0;
        for (int64_t i = threadIdx.x; i < d; i += kBlock) {
          const int32_t v = col[beg + i];
          w += (uint64_t)(row_ptr[v + 1] - row_ptr[v]);
        }
        w = (uint64_t)wave_sum((int64_t)w);
        uint64_t* red = reinterpret_cast<uint64_t*>(big.slot);
        if (lane == 0) red[wave] = w;
        __syncthreads();
        w = red[0] + red[1] + red[2] + red[3];
        w *= weight;
        const uint64_t p = (w + (uint64_t(1) << args.split_shift) - 1) >> args.split_shift;
        parts = p < 2 ? 1 : (p > (uint64_t)kMaxParts ? kMaxParts : (int32_t)p);
      }
      if (threadIdx.x == 0) {
        sched[kSchedParts] = parts;
        sched[kSchedPart] = 0;
        if (parts > 1) {
          int32_t slot = atomicAdd(&st->split_count, 1);
          if (slot < kSplitCap) {
            atomicExch(&args.split[slot].word, ((unsigned long long)parts << 32) | (uint32_t)u);
            const int32_t k = atomicAdd(&args.split[slot].next, 1);
            sched[kSchedPart] = k;
            sched[kSchedEnt] = k < parts ? slot : kNoEntry;
            if (k >= parts) sched[kSchedState] = kStateSkip;  // helpers took every part
          } else {
            sched[kSchedEnt] = kLocalEntry;  // table full: this workgroup takes every part
            sched[kSchedLocalK] = 1;
          }
        }
      }
      __syncthreads();
      if (sched[kSchedState] == kStateSkip) continue;
    }
    const Part pt{sched[kSchedPart], sched[kSchedParts]};
    const uint64_t h = process_source<kWavesPerBlock, K, Wide, OffT>(
        u, beg, d, row_ptr, col, tv, big, ws, kChunk, args.max_kicks, args.force_sorted, la, pt);
    hits += h;
    credit(u, h);
    if (args.src_cnt && h && lane == 0)
      atomicAdd((unsigned long long*)&args.src_cnt[u], (unsigned long long)h);
  }

  const Table mine = table_at<PV>(smem + wave * small_bytes_per_wave(PV), kSmallSide);
  // Wave-mode sources.  With many per wave (large graphs, batches) a wave takes
  // runs of kSmallGrab consecutive list entries -- nearby vertices, which share
  // cache lines -- its first run by its id, later ones from a global cursor, so
  // the waves finish together.  With few per wave (small graphs) the cursor's
  // atomics would come in one burst, so the sources go round robin instead.
  const int32_t waves = (int32_t)gridDim.x * kWavesPerBlock;
  const int32_t w_id = (int32_t)blockIdx.x * kWavesPerBlock + wave;
  const bool dynamic = n_small >= 2 * kSmallGrab * waves;
  int32_t first = dynamic ? w_id * kSmallGrab : w_id;
  while (first < n_small) {
    const int32_t last = dynamic ? (first + kSmallGrab < n_small ? first + kSmallGrab : n_small)
                                 : first + 1;
    // the run's source ids and row bounds, one source per lane, loaded together
    int32_t ru = 0;
    OffT rb = 0, re = 0;
    if (lane < last - first) {
      ru = list[n_large + first + lane];
      rb = row_ptr[ru];
      re = row_ptr[ru + 1];
    }
    for (int32_t i = first; i < last; ++i) {
      const int src = i - first;
      const int32_t u = read_lane(ru, src);
      int64_t beg, d;
      if (sizeof(OffT) == 4) {
        beg = read_lane((int32_t)rb, src);
        d = (int64_t)read_lane((int32_t)re, src) - beg;
      } else {
        beg = read_lane64((int64_t)rb, src);
        d = read_lane64((int64_t)re, src) - beg;
      }
      const uint64_t h = process_source<1, K, Wide, OffT>(u, beg, d, row_ptr, col, tv, mine, ws,
                                                          kSmallMax, args.max_kicks,
                                                          args.force_sorted, la, Part{0, 1});
      hits += h;
      credit(u, h);
      if (args.src_cnt && h && lane == 0)
        atomicAdd((unsigned long long*)&args.src_cnt[u], (unsigned long long)h);
    }
    if (dynamic) {
      int32_t next = 0;
      if (lane == 0) next = waves * kSmallGrab + atomicAdd(&st->small_cursor, kSmallGrab);
      first = first_lane(next);
    } else {
      first += waves;
    }
  }
  if (pend_h && lane == 0)
    atomicAdd((unsigned long long*)&args.totals[pend_g], (unsigned long long)pend_h);
  // the directed kind's sums are per lane
  if (K == kKindDirected) hits = (uint64_t)wave_sum((int64_t)hits);
  if (lane == 0 && hits) atomicAdd((unsigned long long*)total, (unsigned long long)hits);
}

// Graph id of every vertex of a batch: -1 first, then graph g writes its range
// [vtx_off[g], vtx_off[g+1]) clamped to [0, n), so a malformed offset table can
// only leave vertices unattributed, never write out of bounds.
__global__ void graph_map_kernel(int64_t num_graphs, const int64_t* __restrict__ vtx_off, int64_t n,
                                 int32_t* __restrict__ gid) {
  for (int64_t g = blockIdx.x; g < num_graphs; g += gridDim.x) {
    int64_t b = vtx_off[g], e = vtx_off[g + 1];
    b = b < 0 ? 0 : (b > n ? n : b);
    e = e < b ? b : (e > n ? n : e);
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) gid[i] = (int32_t)g;
  }
}

__global__ void fill_i32_kernel(int32_t* p, int64_t len, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = v;
}

struct CountLayout {
  CountState* st;
  SplitEntry* split;
  int32_t* list;
  uint64_t* total_scratch;
  int32_t* gid;  // batched mode only
  size_t bytes;
};

CountLayout carve_count(void* ws, int64_t n, bool batched) {
  Carver c(ws);
  CountLayout L;
  L.st = c.take<CountState>(1);
  L.split = c.take<SplitEntry>(kSplitCap);
  L.list = c.take<int32_t>(n);
  L.total_scratch = c.take<uint64_t>(1);
  L.gid = batched ? c.take<int32_t>(n) : nullptr;
  L.bytes = c.used();
  return L;
}

struct Tune {
  int small_max;
  int force_sorted;
  int blocks_per_cu;  // 0: occupancy limit
  int max_kicks;      // cuckoo placements per key before the stash
  int split_shift;    // log2 of the wedges per part of a split source; 0: never split
};

tc_status read_tune(const tc_tune* tune, Tune* out) {
  out->small_max = kSmallDefault;
  out->force_sorted = 0;
  out->blocks_per_cu = 0;
  out->max_kicks = kMaxKicks;
  out->split_shift = kSplitDefaultLog2;
  if (!tune) return TC_OK;
  if (tune->split_log2 < -1 || tune->split_log2 > 40)
    return fail(TC_ERR_INVALID_ARG, "tc_tune.split_log2 must be in [-1, 40]");
  if (tune->split_log2 == -1) out->split_shift = 0;
  else if (tune->split_log2 > 0) out->split_shift = tune->split_log2;
  if (tune->max_kicks < -1 || tune->max_kicks > 1024)
    return fail(TC_ERR_INVALID_ARG, "tc_tune.max_kicks must be in [-1, 1024]");
  if (tune->max_kicks != 0) out->max_kicks = tune->max_kicks < 0 ? 0 : tune->max_kicks;
  if (tune->small_max != 0) {
    if (tune->small_max < 1 || tune->small_max > kSmallMax)
      return fail(TC_ERR_INVALID_ARG, "tc_tune.small_max must be 0 or in [1, %d]", kSmallMax);
    out->small_max = tune->small_max;
  }
  if (tune->probe != TC_PROBE_AUTO && tune->probe != TC_PROBE_SORTED)
    return fail(TC_ERR_INVALID_ARG, "unknown tc_tune.probe %d", tune->probe);
  out->force_sorted = tune->probe == TC_PROBE_SORTED;
  if (tune->blocks_per_cu < 0 || tune->blocks_per_cu > 64)
    return fail(TC_ERR_INVALID_ARG, "tc_tune.blocks_per_cu must be in [0, 64]");
  out->blocks_per_cu = tune->blocks_per_cu;
  return TC_OK;
}

// Persistent grid of a count kernel instantiation: resident workgroups per CU
// (queried once per device; concurrent first calls store the same value, and
// the per-device slots are atomics so those stores do not race) x CUs.
template <int K, bool Wide, typename OffT>
int count_grid(int blocks_per_cu) {
  static std::atomic<int> cached[64];
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  int occ = cached[dev].load(std::memory_order_relaxed);
  if (occ == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, count_kernel<K, Wide, OffT>, kBlock, 0) !=
            hipSuccess ||
        occ <= 0) {
      occ = 2;
    }
    cached[dev].store(occ, std::memory_order_relaxed);
  }
  const int per_cu = blocks_per_cu > 0 && blocks_per_cu < occ ? blocks_per_cu : occ;
  return per_cu * device_cu_count();
}

CountArgs base_args(const Tune& tune) {
  CountArgs args;
  args.gid = nullptr;
  args.totals = nullptr;
  args.src_cnt = nullptr;
  args.list_status = nullptr;
  args.list = ListArgs{nullptr, nullptr, 0, nullptr};
  args.force_sorted = tune.force_sorted;
  args.max_kicks = tune.max_kicks;
  args.split_shift = tune.split_shift;
  args.split = nullptr;
  args.codes = DirCodes{};
  return args;
}

// The persistent count launch over the binned sources, capped at one workgroup
// per 16 vertices so that a small graph launches a small grid.
template <int K, typename OffT>
void launch_count(int64_t n, const OffT* row_ptr, const int32_t* col, const CountLayout& L,
                  uint64_t* tot, uint64_t* tv, const CountArgs& args_in, const Tune& tune,
                  hipStream_t s) {
  CountArgs args = args_in;
  args.split = L.split;
  const int64_t cap = (n + 15) / 16;
  if (n <= (int64_t(1) << 24)) {
    const int grid = (int)std::min<int64_t>(count_grid<K, false, OffT>(tune.blocks_per_cu), cap);
    count_kernel<K, false, OffT><<<grid, kBlock, 0, s>>>(row_ptr, col, L.list, L.st, tot, tv, args);
  } else {
    const int grid = (int)std::min<int64_t>(count_grid<K, true, OffT>(tune.blocks_per_cu), cap);
    count_kernel<K, true, OffT><<<grid, kBlock, 0, s>>>(row_ptr, col, L.list, L.st, tot, tv, args);
  }
}

template <bool PV, typename OffT>
tc_status count_impl(int64_t n, const OffT* row_ptr, const int32_t* col, uint64_t* total,
                     uint64_t* tv, int64_t num_graphs, const int64_t* vtx_off, uint64_t* totals,
                     const Tune& tune, const CountLayout& L, hipStream_t s) {
  constexpr int K = PV ? kKindPerVertex : kKindTotal;
  uint64_t* tot = total ? total : L.total_scratch;
  CountArgs args = base_args(tune);
  init_state_kernel<<<1, 256, 0, s>>>(L.st, L.split, tot);
  if (PV) zero_u64_kernel<<<grid_for(n, 256, 8192), 256, 0, s>>>(tv, n);
  if (totals) {
    zero_u64_kernel<<<grid_for(num_graphs, 256, 1024), 256, 0, s>>>(totals, num_graphs);
    fill_i32_kernel<<<grid_for(n, 256, 8192), 256, 0, s>>>(L.gid, n, -1);
    if (num_graphs > 0)
      graph_map_kernel<<<grid_for(num_graphs, 1, 8192), 256, 0, s>>>(num_graphs, vtx_off, n, L.gid);
    args.gid = L.gid;
    args.totals = totals;
  }
  if (n > 0) {
    launch_bins<OffT>(n, row_ptr, L.st, L.list, tune.small_max, s);
    launch_count<K, OffT>(n, row_ptr, col, L, tot, tv, args, tune, s);
  }
  return check_hip(hipGetLastError(), "tc_count launch");
}

tc_status check_dag(const tc_csr* dag) {
  if (!dag) return fail(TC_ERR_INVALID_ARG, "dag is NULL");
  if (dag->n < 0) return fail(TC_ERR_INVALID_ARG, "negative n");
  if (dag->n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)dag->n);
  if (dag->offset_bytes != 4 && dag->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", dag->offset_bytes);
  return TC_OK;
}

// Shared front end of the three count entry points.  batched: num_graphs /
// vtx_off / totals are meaningful.
template <bool PV>
tc_status count_dispatch(const tc_csr* dag, uint64_t* total, uint64_t* tv, bool batched,
                         int64_t num_graphs, const int64_t* vtx_off, uint64_t* totals,
                         const tc_tune* tune, void* ws, size_t* ws_bytes, void* stream) {
  tc_status st = check_dag(dag);
  if (st != TC_OK) return st;
  Tune t;
  if ((st = read_tune(tune, &t)) != TC_OK) return st;
  if (batched && (num_graphs < 0 || num_graphs > INT32_MAX))
    return fail(TC_ERR_INVALID_ARG, "num_graphs=%lld out of range", (long long)num_graphs);
  if (workspace_query(ws, ws_bytes, carve_count(nullptr, dag->n, batched).bytes, &st)) return st;
  if (!dag->row_ptr || (PV && dag->n > 0 && !tv) || (!PV && !batched && !total) ||
      (batched && num_graphs > 0 && (!vtx_off || !totals)))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const CountLayout L = carve_count(ws, dag->n, batched);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint64_t* gt = batched && num_graphs > 0 ? totals : nullptr;
  if (dag->offset_bytes == 4)
    st = count_impl<PV, int32_t>(dag->n, static_cast<const int32_t*>(dag->row_ptr), dag->col, total,
                                 tv, num_graphs, vtx_off, gt, t, L, s);
  else
    st = count_impl<PV, int64_t>(dag->n, static_cast<const int64_t*>(dag->row_ptr), dag->col, total,
                                 tv, num_graphs, vtx_off, gt, t, L, s);
  return st == TC_OK ? ok() : st;
}

// ---- listing: per-source counts -> row offsets -> the rows themselves ----------

__global__ void reset_cursors_kernel(CountState* st, uint64_t* total) {
  st->large_cursor = 0;
  st->small_cursor = 0;
  *total = 0;
}

struct SrcLoad {
  const uint64_t* cnt;
  __device__ int64_t operator()(int64_t i) const { return (int64_t)cnt[i]; }
};
struct SrcStore {
  int64_t* off;
  __device__ void operator()(int64_t i, int64_t p) const { off[i] = p; }
};

__global__ void list_finalize_kernel(const int64_t* total, int64_t cap, int64_t* count_out) {
  const int64_t t = *total;
  *count_out = t > cap ? -(int64_t)TC_ERR_CAPACITY : t;
}

struct ListLayout {
  CountLayout c;
  uint64_t* src_cnt;
  int64_t* src_off;
  int64_t* partial;
  size_t bytes;
};

ListLayout carve_list(void* ws, int64_t n) {
  Carver c(ws);
  ListLayout L;
  L.c.st = c.take<CountState>(1);
  L.c.split = c.take<SplitEntry>(kSplitCap);
  L.c.list = c.take<int32_t>(n);
  L.c.total_scratch = c.take<uint64_t>(1);
  L.c.gid = nullptr;
  L.src_cnt = c.take<uint64_t>(n);
  L.src_off = c.take<int64_t>(n);
  L.partial = c.take<int64_t>(scan_partial_len(n));
  L.bytes = c.used();
  L.c.bytes = L.bytes;
  return L;
}

// Pass 1 counts the hits of every source (the same persistent launch as
// tc_count), a scan turns them into row offsets, and pass 2 repeats the
// enumeration writing each hit as a row.  Both passes find exactly the same
// hits per source, so every source writes inside its own range.
template <typename OffT>
tc_status list_impl(int64_t n, const OffT* row_ptr, const int32_t* col, int32_t* out, int64_t cap,
                    int64_t* count_out, const Tune& tune, const ListLayout& L, hipStream_t s) {
  uint64_t* tot = L.c.total_scratch;
  init_state_kernel<<<1, 256, 0, s>>>(L.c.st, L.c.split, tot);
  zero_u64_kernel<<<grid_for(n, 256, 8192), 256, 0, s>>>(L.src_cnt, n);
  if (n > 0) {
    launch_bins<OffT>(n, row_ptr, L.c.st, L.c.list, tune.small_max, s);
    CountArgs a1 = base_args(tune);
    a1.src_cnt = L.src_cnt;
    launch_count<kKindTotal, OffT>(n, row_ptr, col, L.c, tot, nullptr, a1, tune, s);
  }
  hipError_t e = scan_exclusive<OpSum>(n, SrcLoad{L.src_cnt}, SrcStore{L.src_off}, L.partial, s);
  if (e != hipSuccess) return check_hip(e, "listing offset scan");
  list_finalize_kernel<<<1, 1, 0, s>>>(L.partial + scan_num_tiles(n), cap, count_out);
  if (n > 0) {
    reset_cursors_kernel<<<1, 1, 0, s>>>(L.c.st, tot);
    CountArgs a2 = base_args(tune);
    a2.list_status = count_out;
    a2.list = ListArgs{out, L.src_off, cap, nullptr};
    launch_count<kKindList, OffT>(n, row_ptr, col, L.c, tot, nullptr, a2, tune, s);
  }
  return check_hip(hipGetLastError(), "tc_list_triangles launch");
}

// ---- per-edge support ------------------------------------------------------

// m_out = m = row_ptr[n], or -TC_ERR_CAPACITY when it exceeds cap; sup[0, m) = 0.
template <typename OffT>
__global__ void support_init_kernel(const OffT* __restrict__ row_ptr, int64_t n, int64_t cap,
                                    uint32_t* __restrict__ sup, int64_t* __restrict__ m_out) {
  const int64_t m = (int64_t)row_ptr[n];
  if (blockIdx.x == 0 && threadIdx.x == 0) *m_out = m > cap ? -(int64_t)TC_ERR_CAPACITY : m;
  if (m > cap) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) sup[i] = 0;
}

// One count launch with the support kind: every hit adds one to its edge (v, w),
// each (u, v) list adds its hits to (u, v), and each source adds the hits
// counted on w's slot to (u, w).
template <typename OffT>
tc_status support_impl(int64_t n, const OffT* row_ptr, const int32_t* col, uint32_t* sup,
                       int64_t cap, int64_t* m_out, uint64_t* total, const Tune& tune,
                       const CountLayout& L, hipStream_t s) {
  uint64_t* tot = total ? total : L.total_scratch;
  init_state_kernel<<<1, 256, 0, s>>>(L.st, L.split, tot);
  support_init_kernel<OffT><<<grid_for(cap, 256, 8192), 256, 0, s>>>(row_ptr, n, cap, sup, m_out);
  if (n > 0) {
    launch_bins<OffT>(n, row_ptr, L.st, L.list, tune.small_max, s);
    CountArgs args = base_args(tune);
    args.list_status = m_out;
    args.list = ListArgs{nullptr, nullptr, 0, sup};
    launch_count<kKindSupport, OffT>(n, row_ptr, col, L, tot, nullptr, args, tune, s);
  }
  return check_hip(hipGetLastError(), "tc_edge_support launch");
}

// ---- directed queries ----------------------------------------------------------

// The table of a directed query with pair codes q = (p01, p02, p12): for every
// combination of a triangle's direction codes, the one-to-one maps of the query
// nodes onto (u, v, w) = (0, 1, 2) that carry each query arc onto an arc (or,
// induced, whose arcs agree in both directions), divided by the query's
// automorphisms (the maps onto one triangle fall into classes of that size).
DirCodes directed_codes(const int32_t q[3], bool induced) {
  // arc i -> j under the pair codes c (c[0]: 0-1, c[1]: 0-2, c[2]: 1-2; bit 0:
  // lower -> higher, bit 1: higher -> lower)
  auto arc = [](const int32_t c[3], int i, int j) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int32_t code = c[lo == 0 ? hi - 1 : 2];
    return ((code >> (i < j ? 0 : 1)) & 1) != 0;
  };
  static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int aut = 0;
  for (const auto& f : perm) {
    bool keeps = true;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (i != j && arc(q, i, j) != arc(q, f[i], f[j])) keeps = false;
    aut += keeps;
  }
  DirCodes t{};
  for (int c = 0; c < 64; ++c) {
    const int32_t g[3] = {c >> 4, (c >> 2) & 3, c & 3};
    int maps = 0;
    for (const auto& f : perm) {
      bool ok = true;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          if (i == j) continue;
          const bool qa = arc(q, i, j), ga = arc(g, f[i], f[j]);
          if (induced ? qa != ga : (qa && !ga)) ok = false;
        }
      maps += ok;
    }
    t.v[c] = (uint8_t)(maps / aut);
  }
  return t;
}

// The table of a triangle query with edge labels q = (q01, q02, q12): for every
// combination of a triangle's edge labels (codes of (u, v), (u, w), (v, w)),
// the one-to-one maps of the query nodes onto (u, v, w) = (0, 1, 2) that give
// every query edge the label of its image, divided by the permutations of the
// query nodes that keep every edge's label.
DirCodes edge_label_codes(const int32_t q[3]) {
  // label of the edge {i, j} under the pair codes c (c[0]: 0-1, c[1]: 0-2, c[2]: 1-2)
  auto lab = [](const int32_t c[3], int i, int j) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    return c[lo == 0 ? hi - 1 : 2];
  };
  static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int aut = 0;
  for (const auto& f : perm) {
    bool keeps = true;
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j)
        if (lab(q, i, j) != lab(q, f[i], f[j])) keeps = false;
    aut += keeps;
  }
  DirCodes t{};
  for (int c = 0; c < 64; ++c) {
    const int32_t g[3] = {c >> 4, (c >> 2) & 3, c & 3};
    int maps = 0;
    for (const auto& f : perm) {
      bool ok = true;
      for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
          if (lab(g, f[i], f[j]) != lab(q, i, j)) ok = false;
      maps += ok;
    }
    t.v[c] = (uint8_t)(maps / aut);
  }
  return t;
}

// One count launch of the directed kind: every wedge u -> v -> w closed by
// (u, w) adds the table entry of its three direction codes.
template <typename OffT>
tc_status directed_impl(int64_t n, const OffT* row_ptr, const int32_t* col, const uint8_t* dir,
                        const DirCodes& codes, uint64_t* total, const Tune& tune,
                        const CountLayout& L, hipStream_t s) {
  init_state_kernel<<<1, 256, 0, s>>>(L.st, L.split, total);
  if (n > 0) {
    launch_bins<OffT>(n, row_ptr, L.st, L.list, tune.small_max, s);
    CountArgs args = base_args(tune);
    args.codes = codes;
    args.list.dir = dir;
    launch_count<kKindDirected, OffT>(n, row_ptr, col, L, total, nullptr, args, tune, s);
  }
  return check_hip(hipGetLastError(), "tc_count_directed launch");
}

// ---- diamonds: two triangles sharing an edge ---------------------------------

__global__ void diamond_init_kernel(uint64_t* total) { *total = 0; }

// Sum over the edges of C(s, 2), s = the edge's support (m from m_out; nothing
// when it reports an error).  A few workgroups per CU, one atomic each: one per
// wave over thousands of workgroups queued on the total's cache line.
__global__ __launch_bounds__(256) void diamond_reduce_kernel(const uint32_t* __restrict__ sup,
                                                             const int64_t* __restrict__ m_out,
                                                             uint64_t* __restrict__ total) {
  __shared__ uint64_t part[256 / kWave];
  const int64_t m = *m_out;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint64_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint64_t c = sup[i];
    acc += c * (c - 1) / 2;  // 0 for c = 0 and c = 1
  }
  const uint64_t w = (uint64_t)wave_sum((int64_t)acc);
  if (lane_id() == 0) part[threadIdx.x / kWave] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t b = 0;
    for (int i = 0; i < 256 / kWave; ++i) b += part[i];
    if (b) atomicAdd((unsigned long long*)total, (unsigned long long)b);
  }
}

struct DiamondLayout {
  CountLayout c;
  uint32_t* sup;
  size_t bytes;
};

DiamondLayout carve_diamonds(void* ws, int64_t n, int64_t cap) {
  Carver c(ws);
  DiamondLayout L;
  L.c.st = c.take<CountState>(1);
  L.c.split = c.take<SplitEntry>(kSplitCap);
  L.c.list = c.take<int32_t>(n);
  L.c.total_scratch = c.take<uint64_t>(1);
  L.c.gid = nullptr;
  L.sup = c.take<uint32_t>(cap);
  L.bytes = c.used();
  L.c.bytes = L.bytes;
  return L;
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_edge_support(const tc_csr* dag, uint32_t* support, int64_t capacity,
                                     int64_t* m_out, uint64_t* total, const tc_tune* tune,
                                     void* ws, size_t* ws_bytes, void* stream) {
  using namespace tc;
  tc_status st = check_dag(dag);
  if (st != TC_OK) return st;
  Tune t;
  if ((st = read_tune(tune, &t)) != TC_OK) return st;
  if (capacity < 0) return fail(TC_ERR_INVALID_ARG, "negative capacity");
  if (workspace_query(ws, ws_bytes, carve_count(nullptr, dag->n, false).bytes, &st)) return st;
  if (!dag->row_ptr || !m_out || (capacity > 0 && !support))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const CountLayout L = carve_count(ws, dag->n, false);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dag->offset_bytes == 4)
    st = support_impl<int32_t>(dag->n, static_cast<const int32_t*>(dag->row_ptr), dag->col, support,
                               capacity, m_out, total, t, L, s);
  else
    st = support_impl<int64_t>(dag->n, static_cast<const int64_t*>(dag->row_ptr), dag->col, support,
                               capacity, m_out, total, t, L, s);
  return st == TC_OK ? ok() : st;
}

extern "C" tc_status tc_list_triangles(const tc_csr* dag, int32_t* triples, int64_t capacity,
                                       int64_t* count_out, const tc_tune* tune, void* ws,
                                       size_t* ws_bytes, void* stream) {
  using namespace tc;
  tc_status st = check_dag(dag);
  if (st != TC_OK) return st;
  Tune t;
  if ((st = read_tune(tune, &t)) != TC_OK) return st;
  if (capacity < 0) return fail(TC_ERR_INVALID_ARG, "negative capacity");
  if (capacity > ((int64_t)1 << 40))
    return fail(TC_ERR_UNSUPPORTED, "capacity=%lld is beyond 2^40", (long long)capacity);
  if (workspace_query(ws, ws_bytes, carve_list(nullptr, dag->n).bytes, &st)) return st;
  if (!dag->row_ptr || !count_out || (capacity > 0 && !triples))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const ListLayout L = carve_list(ws, dag->n);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dag->offset_bytes == 4)
    st = list_impl<int32_t>(dag->n, static_cast<const int32_t*>(dag->row_ptr), dag->col, triples,
                            capacity, count_out, t, L, s);
  else
    st = list_impl<int64_t>(dag->n, static_cast<const int64_t*>(dag->row_ptr), dag->col, triples,
                            capacity, count_out, t, L, s);
  return st == TC_OK ? ok() : st;
}

extern "C" tc_status tc_count(const tc_csr* dag, uint64_t* total, const tc_tune* tune, void* ws,
                              size_t* ws_bytes, void* stream) {
  return tc::count_dispatch<false>(dag, total, nullptr, false, 0, nullptr, nullptr, tune, ws,
                                   ws_bytes, stream);
}

extern "C" tc_status tc_count_per_vertex(const tc_csr* dag, uint64_t* per_vertex, uint64_t* total,
                                         const tc_tune* tune, void* ws, size_t* ws_bytes,
                                         void* stream) {
  return tc::count_dispatch<true>(dag, total, per_vertex, false, 0, nullptr, nullptr, tune, ws,
                                  ws_bytes, stream);
}

extern "C" tc_status tc_count_batched(const tc_csr* dag, int64_t num_graphs, const int64_t* vtx_off,
                                      uint64_t* totals, uint64_t* per_vertex, uint64_t* total,
                                      const tc_tune* tune, void* ws, size_t* ws_bytes,
                                      void* stream) {
  if (per_vertex)
    return tc::count_dispatch<true>(dag, total, per_vertex, true, num_graphs, vtx_off, totals, tune,
                                    ws, ws_bytes, stream);
  return tc::count_dispatch<false>(dag, total, nullptr, true, num_graphs, vtx_off, totals, tune, ws,
                                   ws_bytes, stream);
}

extern "C" tc_status tc_count_directed(const tc_csr* dag, const uint8_t* dir, int32_t p01,
                                       int32_t p02, int32_t p12, int32_t induced,
                                       uint64_t* total, const tc_tune* tune, void* ws,
                                       size_t* ws_bytes, void* stream) {
  using namespace tc;
  tc_status st = check_dag(dag);
  if (st != TC_OK) return st;
  Tune t;
  if ((st = read_tune(tune, &t)) != TC_OK) return st;
  const int32_t q[3] = {p01, p02, p12};
  for (int32_t c : q)
    if (c < 1 || c > 3)
      return fail(TC_ERR_INVALID_ARG, "pattern codes must be 1, 2 or 3 (every pair joined), got %d",
                  c);
  if (induced != 0 && induced != 1) return fail(TC_ERR_INVALID_ARG, "induced must be 0 or 1");
  if (workspace_query(ws, ws_bytes, carve_count(nullptr, dag->n, false).bytes, &st)) return st;
  if (!dag->row_ptr || !total || (dag->n > 0 && !dir))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const CountLayout L = carve_count(ws, dag->n, false);
  const DirCodes codes = directed_codes(q, induced != 0);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dag->offset_bytes == 4)
    st = directed_impl<int32_t>(dag->n, static_cast<const int32_t*>(dag->row_ptr), dag->col, dir,
                                codes, total, t, L, s);
  else
    st = directed_impl<int64_t>(dag->n, static_cast<const int64_t*>(dag->row_ptr), dag->col, dir,
                                codes, total, t, L, s);
  return st == TC_OK ? ok() : st;
}

// The coded count of an edge-labelled query, for tc_count_edge_labelled (which
// first filters the DAG to the edges whose label is in the query).
namespace tc {

tc_status count_coded_edge_labels(const tc_csr* dag, const uint8_t* edge_labels, const int32_t q[3],
                                  uint64_t* total, const tc_tune* tune, void* ws,
                                  size_t* ws_bytes, void* stream) {
  tc_status st = check_dag(dag);
  if (st != TC_OK) return st;
  Tune t;
  if ((st = read_tune(tune, &t)) != TC_OK) return st;
  for (int i = 0; i < 3; ++i)
    if (q[i] < 0 || q[i] > 3)
      return fail(TC_ERR_INVALID_ARG, "edge labels must be in [0, 3], got %d", q[i]);
  if (workspace_query(ws, ws_bytes, carve_count(nullptr, dag->n, false).bytes, &st)) return st;
  if (!dag->row_ptr || !total || (dag->n > 0 && !edge_labels))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const CountLayout L = carve_count(ws, dag->n, false);
  const DirCodes codes = edge_label_codes(q);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dag->offset_bytes == 4)
    st = directed_impl<int32_t>(dag->n, static_cast<const int32_t*>(dag->row_ptr), dag->col,
                                edge_labels, codes, total, t, L, s);
  else
    st = directed_impl<int64_t>(dag->n, static_cast<const int64_t*>(dag->row_ptr), dag->col,
                                edge_labels, codes, total, t, L, s);
  return st;
}

}  // namespace tc

extern "C" tc_status tc_count_diamonds(const tc_csr* dag, int64_t edge_capacity, uint64_t* total,
                                       int64_t* m_out, const tc_tune* tune, void* ws,
                                       size_t* ws_bytes, void* stream) {
  using namespace tc;
  tc_status st = check_dag(dag);
  if (st != TC_OK) return st;
  Tune t;
  if ((st = read_tune(tune, &t)) != TC_OK) return st;
  if (edge_capacity < 0) return fail(TC_ERR_INVALID_ARG, "negative edge_capacity");
  if (edge_capacity > ((int64_t)1 << 40))
    return fail(TC_ERR_UNSUPPORTED, "edge_capacity=%lld is beyond 2^40", (long long)edge_capacity);
  if (workspace_query(ws, ws_bytes, carve_diamonds(nullptr, dag->n, edge_capacity).bytes, &st))
    return st;
  if (!dag->row_ptr || !total || !m_out) return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const DiamondLayout L = carve_diamonds(ws, dag->n, edge_capacity);
  hipStream_t s = static_cast<hipStream_t>(stream);
  diamond_init_kernel<<<1, 1, 0, s>>>(total);
  if (dag->offset_bytes == 4)
    st = support_impl<int32_t>(dag->n, static_cast<const int32_t*>(dag->row_ptr), dag->col, L.sup,
                               edge_capacity, m_out, nullptr, t, L.c, s);
  else
    st = support_impl<int64_t>(dag->n, static_cast<const int64_t*>(dag->row_ptr), dag->col, L.sup,
                               edge_capacity, m_out, nullptr, t, L.c, s);
  if (st != TC_OK) return st;
  diamond_reduce_kernel<<<grid_for(edge_capacity, 256, 4 * device_cu_count()), 256, 0, s>>>(
      L.sup, m_out, total);
  return check_hip(hipGetLastError(), "tc_count_diamonds launch") == TC_OK ? ok() : TC_ERR_HIP;
}

// ---- per-vertex count without a caller workspace ------------------------------
//
// The workspace of tc_count_per_vertex (class counters, the binned source list,
// a scratch total) lives in one file-scope device array instead.  Host code
// never passes the array's name to a kernel: its device address is taken once
// per device with hipGetSymbolAddress and kept below.

namespace tc {
namespace {

constexpr int64_t kNoAllocMaxVertices = int64_t(1) << 22;
// carve_count(nullptr, kNoAllocMaxVertices, false).bytes, checked on every call
constexpr size_t kNoAllocBytes =
    (size_t(4) << 22) + kSplitCap * sizeof(SplitEntry) + 1024;

static __device__ __align__(256) char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {nullptr};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
tc_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(TC_ERR_UNSUPPORTED, "device %d beyond 64 devices", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return check_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(TC_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TC_OK;
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_count_per_vertex_noalloc(const tc_csr* dag, uint64_t* per_vertex,
                                                 uint64_t* total, const tc_tune* tune,
                                                 void* stream) {
  using namespace tc;
  tc_status st = check_dag(dag);
  if (st != TC_OK) return st;
  if (dag->n > kNoAllocMaxVertices)
    return fail(TC_ERR_CAPACITY, "n=%lld is above the %lld vertices the static scratch holds",
                (long long)dag->n, (long long)kNoAllocMaxVertices);
  const size_t need = carve_count(nullptr, dag->n, false).bytes;
  if (need > kNoAllocBytes)
    return fail(TC_ERR_CAPACITY, "scratch of %zu bytes is below the required %zu", kNoAllocBytes,
                need);
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != TC_OK) return st;
  size_t ws_bytes = kNoAllocBytes;
  return count_dispatch<true>(dag, total, per_vertex, false, 0, nullptr, nullptr, tune, ws,
                              &ws_bytes, stream);
}
