// clique4.hip - tc_count_k4: the 4-clique query, the next clique after the
// triangle in the paper's subgraph-matching view (Sec. II-A; Alg. 1 matches a
// query by advancing one query node per iteration under the unique mapping
// order).  On the oriented graph every 4-clique appears once as u -> v -> w -> x
// with all six edges present: v in N+(u), w in S = N+(u) & N+(v), x in
// N+(w) & S.  Look-ahead (Sec. III-C): a source needs d+(u) >= 3, a second node
// d+(v) >= 2, a third node d+(w) >= 1.
//
// A workgroup takes runs of kGrab sources from a global cursor, one source at a
// time; N+(u) sits in LDS when it has at most kLdsKeys ids: in a cuckoo table
// up to kHashKeys ids, else sorted.  Its four waves take the v round robin.
// Sources whose wedge work sum_v d+(v) exceeds kPartWork are split first into
// up to kMaxParts parts (part k takes every parts-th group of four middles),
// listed as tasks and taken one per claim before the other sources: a heavy
// source's middles then run on several workgroups instead of setting the
// launch's tail on one.
//
// For each (u, v) a wave streams N+(v), finds each w in N+(u) and keeps it in
// a per-wave list (S = the kept w); then it walks the N+(w) of 64 kept w at a
// time as one concatenation (one round trip for their row bounds) and counts
// the x that are in S.  With the table, S is also a per-wave bit beside each
// slot, so x is tested by its table probe and that bit; with the sorted copy,
// by binary search in S.  Longer sources keep N+(u) in memory: w and x are
// then tested by binary search in the sorted rows of u and v, and the kept w
// go through a bounded list in chunks.
#include "tc_device.h"
#include "tc_hash.h"
#include "tc_host.h"

#include <algorithm>

namespace tc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kLdsKeys = 2048;           // N+(u) ids held in LDS
constexpr int kListCap = 1024;           // kept w per chunk in the in-memory path
constexpr int kGrab = 4;                 // sources per claim from the global cursor
constexpr int32_t kWalkMax = 1 << 24;    // longest N+(w) walked in a concatenation of 64
constexpr int kHashKeys = 816;           // d+(u) up to which N+(u) goes into an LDS cuckoo table
constexpr int kMaxKicks = 48;
static_assert(kHashKeys <= kListCap, "a hashed source's kept w fit the per-wave list");

// log2 of the slots per half for `keys` keys: load <= 0.4 over both halves.
__host__ __device__ constexpr int k4_side_log2(int keys) {
  const int want = keys + (keys >> 2) + 1;
  int b = 4;
  while ((1 << b) < want) ++b;
  return b;
}
static_assert(2 * (1 << k4_side_log2(kHashKeys)) <= kLdsKeys, "the table fits the key array");

constexpr int64_t kPartWork = 8192;      // wedges sum_v d+(v) per part of a split source
constexpr int kMaxParts = 64;
static_assert(kMaxParts < 65536, "part numbers fit the 16-bit task fields");

struct K4State {
  int32_t cursor;        // runs of kGrab sources (the unsplit ones)
  int32_t task_cursor;   // the split sources' tasks, one per claim
  uint64_t tasks;        // task entries reserved (may pass the capacity)
};

// One part of a split source: its middles iv with (iv / kWavesPerBlock) % parts
// == part.  u = -1 marks an entry of a reservation that did not fit.
struct K4Task {
  int32_t u;
  uint16_t part;
  uint16_t parts;
};

// Task entries of the workspace for n sources.
__host__ __device__ constexpr int64_t k4_task_cap(int64_t n) { return n / 2 + 4096; }

__global__ void k4_init_kernel(K4State* st, uint64_t* total) {
  st->cursor = 0;
  st->task_cursor = 0;
  st->tasks = 0;
  *total = 0;
}

// One wave per source: w = sum of d+(v) over N+(u) with d+(v) >= 2 (the N+(v)
// that the 4-clique walk streams); a source with d+(u) >= 3 and w > kPartWork
// gets ceil(w / kPartWork) tasks (at most kMaxParts, at most one per group of
// four middles) and is marked in split[] so the run cursor skips it.  A wave
// holds up to 64 such sources (lane j the j-th) and reserves their tasks with
// one atomic add, in lane order: one counter shared by every heavy source
// would serialise its atomics.  A source whose tasks do not fit the array
// stays whole and blanks the entries of its reservation below the capacity.
template <typename OffT>
__global__ __launch_bounds__(256) void k4_split_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       K4State* __restrict__ st,
                                                       uint8_t* __restrict__ split,
                                                       K4Task* __restrict__ tasks, int64_t cap) {
  const int lane = lane_id();
  const int64_t per_block = blockDim.x / kWave;
  const int64_t waves = (int64_t)gridDim.x * per_block;
  int64_t held_u = 0;  // lane j < held: the j-th held source and its parts
  int32_t held_p = 0;
  int held = 0;        // uniform
  for (int64_t u = (int64_t)blockIdx.x * per_block + threadIdx.x / kWave;; u += waves) {
    const bool more = u < n;
    if (more) {
      const int64_t ub = row_ptr[u];
      const int64_t du = (int64_t)row_ptr[u + 1] - ub;
      int64_t w = 0;
      if (du >= 3) {
        for (int64_t j = lane; j < du; j += kWave) {
          const int32_t v = col[ub + j];
          const int64_t dv = (int64_t)row_ptr[v + 1] - (int64_t)row_ptr[v];
          w += dv >= 2 ? dv : 0;
        }
      }
      w = wave_sum(w);
      int64_t parts = (w + kPartWork - 1) / kPartWork;
      const int64_t groups = (du + kWavesPerBlock - 1) / kWavesPerBlock;
      parts = parts < kMaxParts ? parts : kMaxParts;
      parts = parts < groups ? parts : groups;
      if (du >= 3 && parts > 1) {
        if (lane == held) {
          held_u = u;
          held_p = (int32_t)parts;
        }
        ++held;
      } else if (lane == 0) {
        split[u] = 0;
      }
    }
    if (held == kWave || (!more && held > 0)) {
      const int32_t incl = wave_inclusive_sum32(held_p);
      const int32_t sum = read_lane(incl, kWave - 1);
      uint64_t base = 0;
      if (lane == 0) base = atomicAdd((unsigned long long*)&st->tasks, (unsigned long long)sum);
      base = (uint64_t)read_lane64((int64_t)base, 0);
      if (lane < held) {
        const uint64_t at = base + (uint64_t)(incl - held_p);
        const bool fits = at + (uint64_t)held_p <= (uint64_t)cap;
        for (int32_t k = 0; k < held_p; ++k) {
          if (fits)
            tasks[at + k] = K4Task{(int32_t)held_u, (uint16_t)k, (uint16_t)held_p};
          else if (at + k < (uint64_t)cap)
            tasks[at + k].u = -1;
        }
        split[held_u] = fits ? 1 : 0;
      }
      held = 0;
      held_p = 0;
    }
    if (!more) break;
  }
}

// Position of w in the sorted keys[0, n), or -1 (keys in LDS or memory).
__device__ __forceinline__ int32_t find_pos(const int32_t* keys, int32_t n, int32_t w) {
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

// Whether x is one of the kept w: keys tkeys[lpos[0..ns)], ascending (the kept
// positions are appended in list order and N+(u), N+(v) are sorted).
__device__ __forceinline__ bool in_kept(const int32_t* tkeys, const uint16_t* lpos, int32_t ns,
                                        int32_t x) {
  int32_t lo = 0, len = ns;
  while (len > 0) {
    const int32_t half = len >> 1;
    if (tkeys[lpos[lo + half]] < x) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo < ns && tkeys[lpos[lo]] == x;
}

// Whether x is in the wave's S: x is a key of the table and its slot carries
// the wave's bit.
__device__ __forceinline__ bool in_wave_set(const int32_t* tkeys, const uint32_t* sbits, int side,
                                            int shift, uint32_t my_bit, int32_t x) {
  const uint32_t hp = hash_product(hash_input<true>(x));
  const uint32_t sa = slot_a_of(hp, shift);
  const uint32_t sb = (uint32_t)side + slot_b_of(hp, shift);
  const int32_t s = tkeys[sa] == x ? (int32_t)sa : (tkeys[sb] == x ? (int32_t)sb : -1);
  return s >= 0 && ((sbits[s >> 3] >> ((s & 7) * 4)) & my_bit) != 0;
}

// Shared memory of one 4-clique workgroup.
struct K4Lds {
  int32_t tkeys[kLdsKeys];
  // per-wave kept list: positions in N+(u) (< kLdsKeys, 16-bit) in the LDS path,
  // ids of w (32-bit, kListCap per chunk) in the in-memory path; 4 KB either way
  int32_t list[kWavesPerBlock][kListCap];
  int32_t segs[kWavesPerBlock][kWave];
  // table path: bit `wave` of a slot's 4-bit field is set while the slot's key is
  // in that wave's S (eight slots per 32-bit word, set and cleared atomically)
  uint32_t sbits[kLdsKeys / 8];
  int64_t next;
  int32_t kfail;
};
static_assert(kLdsKeys <= 65536 && kLdsKeys * 2 <= kListCap * 4, "kept positions fit the list");

// The 4-cliques u -> v -> w -> x of source u whose middle v is in this
// workgroup's part: middles iv with (iv / kWavesPerBlock) % parts == part, so
// wave g takes iv = (part + j parts) kWavesPerBlock + g.  Returns this wave's
// count (uniform across the wave).  Every thread of the workgroup calls it with
// the same arguments (it holds workgroup barriers).
template <typename OffT>
__device__ uint64_t k4_source(int64_t u, int32_t part, int32_t parts,
                              const OffT* __restrict__ row_ptr, const int32_t* __restrict__ col,
                              K4Lds& lds) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  int32_t* tkeys = lds.tkeys;
  uint32_t* sbits = lds.sbits;
  int32_t& kfail = lds.kfail;
  int32_t* lst = lds.list[wave];                                   // in-memory path: ids
  uint16_t* lpos = reinterpret_cast<uint16_t*>(lds.list[wave]);    // LDS path: positions
  int32_t* seg = lds.segs[wave];
  uint64_t found = 0;
  const int64_t ub = row_ptr[u];
  const int32_t du = (int32_t)((int64_t)row_ptr[u + 1] - ub);
  const bool in_lds = du <= kLdsKeys;
  if (du >= 3) {
    const int32_t* urow = col + ub;
    // N+(u) up to kHashKeys ids goes into a two-choice cuckoo table (tc_hash.h's
    // hashes, two halves of `side` slots in tkeys); longer rows, or a table whose
    // insertion fails, are copied sorted for binary search
    bool hashed = du <= kHashKeys;
    const int b = k4_side_log2(du);
    const int side = 1 << b, shift = 32 - b;
    if (hashed) {
      for (int i = threadIdx.x; i < 2 * side; i += kBlock) tkeys[i] = -1;
      for (int i = threadIdx.x; i < (2 * side + 7) / 8; i += kBlock) sbits[i] = 0u;
      if (threadIdx.x == 0) kfail = 0;
      __syncthreads();
      for (int i = threadIdx.x; i < du; i += kBlock) {
        int32_t cur = urow[i];
        int hs = 0;
        for (int kick = 0; kick < kMaxKicks && cur != -1; ++kick) {
          const uint32_t sl = hs ? (uint32_t)side + hash_b<true>(cur, shift)
                                 : hash_a<true>(cur, shift);
          cur = atomicExch(&tkeys[sl], cur);
          hs ^= 1;
        }
        if (cur != -1) kfail = 1;
      }
      __syncthreads();
      hashed = kfail == 0;
      __syncthreads();
    }
    if (in_lds && !hashed)
      for (int i = threadIdx.x; i < du; i += kBlock) tkeys[i] = urow[i];
    __syncthreads();
    const uint32_t my_bit = 1u << wave;
    for (int32_t iv = part * kWavesPerBlock + wave; iv < du; iv += parts * kWavesPerBlock) {
      const int32_t v = (in_lds && !hashed) ? tkeys[iv] : urow[iv];
      const int64_t vb = row_ptr[v];
      const int32_t dv = (int32_t)((int64_t)row_ptr[v + 1] - vb);
      if (dv < 2) continue;
      // stream N+(v): keep the w that are also in N+(u)
      int32_t ns = 0;
      for (int32_t base = 0; base < dv; base += kWave) {
        const int32_t j = base + lane;
        int32_t pos = -1;
        int32_t w = 0;
        if (j < dv) {
          w = col[vb + j];
          if (hashed) {
            // pos: w's slot in the table
            const uint32_t hp = hash_product(hash_input<true>(w));
            const uint32_t sa = slot_a_of(hp, shift);
            const uint32_t sb = (uint32_t)side + slot_b_of(hp, shift);
            pos = tkeys[sa] == w ? (int32_t)sa : (tkeys[sb] == w ? (int32_t)sb : -1);
            if (pos >= 0) atomicOr(&sbits[pos >> 3], my_bit << ((pos & 7) * 4));
          } else {
            pos = in_lds ? find_pos(tkeys, du, w) : find_pos(urow, du, w);
          }
        }
        const uint64_t hit = ballot(pos >= 0);
        if (pos >= 0) {
          if (in_lds) {
            lpos[ns + rank_below(hit)] = (uint16_t)pos;  // a slot, or a sorted position
          } else {
            lst[ns + rank_below(hit)] = w;
          }
        }
        ns += popc(hit);
        // the in-memory path flushes a full chunk (the next 64 could overflow it)
        const bool flush = !in_lds && (ns > kListCap - kWave || base + kWave >= dv);
        if (!in_lds && !flush) continue;
        if (!in_lds) {
          wave_sync();
          for (int32_t a = 0; a < ns; ++a) {
            const int32_t ww = lst[a];
            const int64_t wb = row_ptr[ww];
            const int32_t dw = (int32_t)((int64_t)row_ptr[ww + 1] - wb);
            for (int32_t xb = 0; xb < dw; xb += kWave) {
              bool ok = false;
              if (xb + lane < dw) {
                const int32_t x = col[wb + xb + lane];
                ok = find_pos(urow, du, x) >= 0 && find_pos(col + vb, dv, x) >= 0;
              }
              found += popc(ballot(ok));
            }
          }
          wave_sync();
          ns = 0;
        }
      }
      if (!in_lds) continue;
      if (ns < 2) {
        if (hashed && ns == 1 && lane == 0)
          atomicAnd(&sbits[lpos[0] >> 3], ~(my_bit << ((lpos[0] & 7) * 4)));
        wave_sync();
        continue;
      }
      wave_sync();
      // The x in N+(w) that are kept w themselves, for the kept w 64 at a
      // time: lane a takes w = kept[a0 + a] (one round trip for the row bounds of
      // all 64), and the wave walks the concatenation of their lists 64 positions
      // per step.  Each position's list is the last lane whose list starts at or
      // before it: the starts in the window are marked in LDS and a wave max-scan
      // carries them forward (the marker array holds -1 between steps).
      for (int32_t a0 = 0; a0 < ns; a0 += kWave) {
        int64_t wb = 0;
        int32_t dw = 0;
        if (a0 + lane < ns) {
          const int32_t ww = tkeys[lpos[a0 + lane]];
          wb = row_ptr[ww];
          dw = (int32_t)((int64_t)row_ptr[ww + 1] - wb);
        }
        if (ballot(dw > kWalkMax) != 0) {
          // a list too long for 32-bit positions in the concatenation: one at a time
          for (int a = 0; a < kWave && a0 + a < ns; ++a) {
            const int64_t b1 = read_lane64(wb, a);
            const int32_t d1 = read_lane(dw, a);
            for (int32_t xb = 0; xb < d1; xb += kWave) {
              bool ok = false;
              if (xb + lane < d1) {
                const int32_t x = col[b1 + xb + lane];
                ok = hashed ? in_wave_set(tkeys, sbits, side, shift, my_bit, x)
                            : in_kept(tkeys, lpos, ns, x);
              }
              found += popc(ballot(ok));
            }
          }
          continue;
        }
        const int32_t incl = wave_inclusive_sum32(dw);
        const int32_t start = incl - dw;
        const int32_t total_x = read_lane(incl, kWave - 1);
        // walk position pos of lane a's list is col[pos + delta(a)]; with 32-bit
        // offsets wb < 2^31 and start <= total_x < 2^31, so delta fits OffT
        const OffT delta = (OffT)(wb - start);
        int32_t carry = -1;
        for (int32_t base = 0; base < total_x; base += kWave) {
          const bool marks_here = dw > 0 && start >= base && start < base + kWave;
          if (marks_here) seg[start - base] = lane;
          wave_sync();
          int32_t sk = wave_inclusive_max32(seg[lane]);
          sk = sk > carry ? sk : carry;
          carry = read_lane(sk, kWave - 1);
          wave_sync();
          if (marks_here) seg[start - base] = -1;
          const int32_t src = sk < 0 ? 0 : sk;
          const int64_t at = (int64_t)(base + lane) + (int64_t)__shfl(delta, src, kWave);
          bool ok = false;
          if (base + lane < total_x) {  // then start(src) <= base + lane < start(src) + dw(src)
            const int32_t x = col[at];
            ok = hashed ? in_wave_set(tkeys, sbits, side, shift, my_bit, x)
                        : in_kept(tkeys, lpos, ns, x);
          }
          found += popc(ballot(ok));
        }
      }
      if (hashed) {
        // this wave's bits back to 0 for its next middle
        for (int32_t a = lane; a < ns; a += kWave)
          atomicAnd(&sbits[lpos[a] >> 3], ~(my_bit << ((lpos[a] & 7) * 4)));
      }
      wave_sync();  // the list is rewritten by this wave's next middle
    }
  }
  return found;
}

template <typename OffT>
__global__ __launch_bounds__(kBlock) void k4_kernel(int64_t n, const OffT* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    K4State* __restrict__ st,
                                                    const uint8_t* __restrict__ split,
                                                    const K4Task* __restrict__ tasks,
                                                    int64_t cap, uint64_t* __restrict__ total) {
  __shared__ K4Lds lds;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  lds.segs[wave][lane] = -1;
  uint64_t found = 0;
  // the split sources' parts first, one task per claim
  const int64_t ntask = (int64_t)(st->tasks < (uint64_t)cap ? st->tasks : (uint64_t)cap);
  for (;;) {
    if (threadIdx.x == 0) lds.next = atomicAdd(&st->task_cursor, 1);
    __syncthreads();
    const int64_t t = lds.next;
    __syncthreads();
    if (t >= ntask) break;
    const K4Task task = tasks[t];
    if (task.u >= 0) found += k4_source<OffT>(task.u, task.part, task.parts, row_ptr, col, lds);
    __syncthreads();
  }
  // then runs of kGrab sources, skipping the split ones
  if (threadIdx.x == 0) lds.next = atomicAdd(&st->cursor, 1);
  __syncthreads();
  int64_t u0 = lds.next * kGrab;
  __syncthreads();
  while (u0 < n) {
    for (int64_t u = u0; u < u0 + kGrab && u < n; ++u) {
      if (split[u]) continue;
      found += k4_source<OffT>(u, 0, 1, row_ptr, col, lds);
      __syncthreads();
    }
    if (threadIdx.x == 0) lds.next = atomicAdd(&st->cursor, 1);
    __syncthreads();
    u0 = lds.next * kGrab;
    __syncthreads();
  }
  if (lane == 0 && found) atomicAdd((unsigned long long*)total, (unsigned long long)found);
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_count_k4(const tc_csr* dag, uint64_t* total, void* ws, size_t* ws_bytes,
                                 void* stream) {
  using namespace tc;
  if (!dag) return fail(TC_ERR_INVALID_ARG, "dag is NULL");
  const int64_t n = dag->n;
  if (n < 0) return fail(TC_ERR_INVALID_ARG, "negative n");
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (dag->offset_bytes != 4 && dag->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", dag->offset_bytes);
  const int64_t cap = k4_task_cap(n);
  Carver c0(nullptr);
  (void)c0.take<K4State>(1);
  (void)c0.take<uint8_t>(n);
  (void)c0.take<K4Task>(cap);
  tc_status st;
  if (workspace_query(ws, ws_bytes, c0.used(), &st)) return st;
  if (!dag->row_ptr || !total) return fail(TC_ERR_INVALID_ARG, "null device pointer");
  Carver c(ws);
  K4State* state = c.take<K4State>(1);
  uint8_t* split = c.take<uint8_t>(n);
  K4Task* tasks = c.take<K4Task>(cap);
  hipStream_t s = static_cast<hipStream_t>(stream);
  k4_init_kernel<<<1, 1, 0, s>>>(state, total);
  if (n > 0) {
    const int64_t split_grid =
        std::max<int64_t>(1, std::min<int64_t>((n + kWavesPerBlock - 1) / kWavesPerBlock,
                                               (int64_t)device_cu_count() * 8));
    if (dag->offset_bytes == 4)
      k4_split_kernel<int32_t><<<(int)split_grid, kBlock, 0, s>>>(
          n, static_cast<const int32_t*>(dag->row_ptr), dag->col, state, split, tasks, cap);
    else
      k4_split_kernel<int64_t><<<(int)split_grid, kBlock, 0, s>>>(
          n, static_cast<const int64_t*>(dag->row_ptr), dag->col, state, split, tasks, cap);
    int per_cu = 0;
    if (dag->offset_bytes == 4)
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k4_kernel<int32_t>, kBlock, 0);
    else
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k4_kernel<int64_t>, kBlock, 0);
    const int grid = (int)std::max<int64_t>(
        1, std::min<int64_t>((int64_t)std::max(per_cu, 1) * device_cu_count(), n));
    if (dag->offset_bytes == 4)
      k4_kernel<int32_t><<<grid, kBlock, 0, s>>>(n, static_cast<const int32_t*>(dag->row_ptr),
                                                 dag->col, state, split, tasks, cap, total);
    else
      k4_kernel<int64_t><<<grid, kBlock, 0, s>>>(n, static_cast<const int64_t*>(dag->row_ptr),
                                                 dag->col, state, split, tasks, cap, total);
  }
  st = check_hip(hipGetLastError(), "tc_count_k4 launch");
  return st == TC_OK ? ok() : st;
}
