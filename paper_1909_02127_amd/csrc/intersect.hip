// intersect.hip - tc_segmented_intersect: the segmented-intersection operator
// (Sec. II-B lists it beside advance, filter and compute) applied to triangle
// counting: for every oriented edge (u, v) the sorted lists N+(u) and N+(v) are
// intersected; each common out-neighbour w closes the triangle u -> v -> w, and
// under the unique mapping order every triangle is found once, at its lowest
// edge.  This is the edge-centric alternative to the wedge probe of count.hip.
//
// Load balance is a segmented merge path over the whole graph.  Edge e = (u, v)
// owns a stretch of the merge space of length d+(u) + d+(v) (0 when d+(u) < 2
// or d+(v) = 0: the look-ahead of Sec. III-C), and an exclusive scan P lays the
// stretches end to end.  The merge space is cut into chunks of kLaneSteps merge
// steps, 64 consecutive chunks per wave, and every wave takes one contiguous
// run of those spans.  A lane finds its edge by a search of P, its place in
// that edge's merge by the merge-path diagonal search, and merges one element
// per step from elements staged in LDS kSteps at a time (each round's loads in
// flight at once; a round continues from the heads the last one left, so the
// search is paid once per edge and chunk), moving on to the next edge with a
// non-empty stretch at a stretch's end.  Ties take A = N+(u) first, and a match is counted when A[i]
// is taken while B = N+(v)'s head equals it, so each common neighbour is found
// exactly once, in the chunk that takes A[i].
//
// Per-edge support adds one to (u, v), to (u, w) at A's position and to (v, w)
// at B's position for every match.
#include "tc_device.h"
#include "tc_host.h"
#include "tc_scan.h"

#include <algorithm>

namespace tc {
namespace {

constexpr int kBlock = 256;
constexpr int kSteps = 8;   // merge steps per staging round
constexpr int kRounds = 8;   // staging rounds per lane chunk
constexpr int64_t kLaneSteps = (int64_t)kSteps * kRounds;  // merge steps per lane and span
constexpr int64_t kSpan = (int64_t)kWave * kLaneSteps;      // merge steps per wave and span
constexpr int32_t kPastEnd = INT32_MAX;            // head of an exhausted list (ids < 2^31 - 1)

// Source of every edge and the length of its stretch; stretches past m are 0.
// One wave per source (rows are walked 64 entries at a time).
template <typename OffT>
__global__ __launch_bounds__(256) void edge_work_kernel(int64_t n, const OffT* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        int64_t cap, int32_t* __restrict__ src_of,
                                                        uint32_t* __restrict__ work,
                                                        int64_t* __restrict__ m_out) {
  const int64_t m = (int64_t)rp[n];
  if (blockIdx.x == 0 && threadIdx.x == 0) *m_out = m > cap ? -(int64_t)TC_ERR_CAPACITY : m;
  if (m > cap) return;
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  for (int64_t u = gw; u < n; u += nwaves) {
    const int64_t beg = (int64_t)rp[u];
    const int64_t du = (int64_t)rp[u + 1] - beg;
    for (int64_t i = lane; i < du; i += kWave) {
      const int64_t e = beg + i;
      const int32_t v = col[e];
      const int64_t dv = (int64_t)rp[v + 1] - (int64_t)rp[v];
      src_of[e] = (int32_t)u;
      work[e] = du >= 2 && dv >= 1 ? (uint32_t)(du + dv) : 0u;
    }
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = m + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cap; e += stride)
    work[e] = 0u;
}

struct WorkLoad {
  const uint32_t* work;
  __device__ int64_t operator()(int64_t i) const { return (int64_t)work[i]; }
};
struct PrefixStore {
  int64_t* p;
  __device__ void operator()(int64_t i, int64_t x) const { p[i] = x; }
};

// P[cap] = the grand total S; the support array is cleared to m entries.
__global__ void intersect_finish_scan_kernel(const int64_t* __restrict__ partial, int64_t tiles,
                                             int64_t cap, int64_t* __restrict__ P) {
  P[cap] = tiles > 0 ? partial[tiles] : 0;
}

__global__ void intersect_init_kernel(uint64_t* total) { *total = 0; }

__global__ void clear_u32_kernel(uint32_t* __restrict__ p, const int64_t* __restrict__ m_out) {
  const int64_t m = *m_out;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) p[i] = 0u;
}

// First index in [lo, hi) with P[idx] > x, or hi.
__device__ __forceinline__ int64_t upper_bound(const int64_t* __restrict__ P, int64_t lo, int64_t hi,
                                               int64_t x) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (P[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The same, probing lo, lo + 1, lo + 3, lo + 7, ... first (the answer is
// usually close to lo), then a binary search inside the last gap.
__device__ __forceinline__ int64_t gallop_upper(const int64_t* __restrict__ P, int64_t lo,
                                                int64_t hi, int64_t x) {
  int64_t step = 1, prev = lo;
  int64_t at = lo;
  while (at < hi && P[at] <= x) {
    prev = at + 1;
    at = lo + step * 2 - 1;
    step *= 2;
  }
  return upper_bound(P, prev, at < hi ? at : hi, x);
}

// Element i of the column array by a 32-bit offset from its (uniform) base.
__device__ __forceinline__ int32_t list_at(const int32_t* __restrict__ col, uint32_t i) {
  return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(col) + (uint64_t)i * 4u);
}

template <bool Support, bool Narrow, typename OffT>
__global__ __launch_bounds__(kBlock, 4) void merge_kernel(int64_t cap, const OffT* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ src_of,
                                                     const int64_t* __restrict__ P,
                                                     const int64_t* __restrict__ m_out,
                                                     uint64_t* __restrict__ total,
                                                     uint32_t* __restrict__ sup) {
  __shared__ int32_t stage_all[(kBlock / kWave) * 2 * (kSteps + 1) * kWave];
  if (*m_out < 0) return;
  const int64_t S = P[cap];
  const int lane = lane_id();
  // this lane's staging slots: slot t of A at sa[t * kWave], of B at sb[t * kWave]
  int32_t* const sa = stage_all + (threadIdx.x / kWave) * 2 * (kSteps + 1) * kWave + lane;
  int32_t* const sb = sa + (kSteps + 1) * kWave;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  const int64_t gw = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  // this wave's contiguous run of spans
  const int64_t spans = (S + kSpan - 1) / kSpan;
  const int64_t per = (spans + nwaves - 1) / nwaves;
  const int64_t s_beg = gw * per;
  const int64_t s_end = s_beg + per < spans ? s_beg + per : spans;
  uint64_t hits = 0;
  int64_t e_lo = 0;
  bool first = true;
  for (int64_t sp = s_beg; sp < s_end; ++sp) {
    const int64_t base = sp * kSpan;
    const int64_t last = (base + kSpan < S ? base + kSpan : S) - 1;
    // the span's edge range [e_lo, e_hi] (uniform across the wave)
    e_lo = (first ? upper_bound(P, 0, cap + 1, base) : gallop_upper(P, e_lo, cap + 1, base)) - 1;
    first = false;
    const int64_t e_hi = gallop_upper(P, e_lo, cap + 1, last) - 1;
    int64_t p = base + (int64_t)lane * kLaneSteps;
    if (p > last) continue;
    const int64_t pend = p + kLaneSteps <= last + 1 ? p + kLaneSteps : last + 1;
    int64_t e = upper_bound(P, e_lo, e_hi + 2, p) - 1;
    while (true) {
      const int64_t pe = P[e];
      const int64_t pe1 = P[e + 1];
      const int32_t u = src_of[e];
      const int32_t v = col[e];
      const int64_t ab = (int64_t)rp[u];
      const int64_t a = (int64_t)rp[u + 1] - ab;
      const int64_t bb = (int64_t)rp[v];
      const int64_t b = (int64_t)rp[v + 1] - bb;
      // merge-path diagonal k: i elements of A and k - i of B come first
      const int64_t k = p - pe;
      int64_t lo = k - b > 0 ? k - b : 0;
      int64_t hi = k < a ? k : a;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[ab + mid] <= col[bb + k - mid - 1]) lo = mid + 1;
        else hi = mid;
      }
      int64_t i = lo, j = k - lo;
      const int64_t stop = pend < pe1 ? pend : pe1;
      uint32_t cuv = 0;
      // The steps [p, stop) of this edge, kSteps per round: a round stages the elements
      // its q steps can take, A[i, i + q] and B[j, j + q] (past a list's end: kPastEnd), in
      // this lane's LDS slots, then merges from there; the next round continues from the
      // heads the last one left, with no second search.  The loads take indices clamped
      // to the list (a, b >= 1), so all of a round's loads are in flight together.
      while (p < stop) {
        const int q = (int)(stop - p < kSteps ? stop - p : kSteps);  // 1..kSteps
        {
          int32_t ra[kSteps + 1], rb[kSteps + 1];
          if (Narrow) {
            // column indices below 2^30: 32-bit offsets from the (uniform) column base
            const uint32_t x0 = (uint32_t)(ab + i), xl = (uint32_t)(ab + a - 1);
            const uint32_t y0 = (uint32_t)(bb + j), yl = (uint32_t)(bb + b - 1);
#pragma unroll
            for (int t = 0; t <= kSteps; ++t) {
              ra[t] = list_at(col, x0 + t < xl ? x0 + t : xl);
              rb[t] = list_at(col, y0 + t < yl ? y0 + t : yl);
            }
          } else {
#pragma unroll
            for (int t = 0; t <= kSteps; ++t) {
              const int64_t x = i + t, y = j + t;
              ra[t] = col[ab + (x < a ? x : a - 1)];
              rb[t] = col[bb + (y < b ? y : b - 1)];
            }
          }
#pragma unroll
          for (int t = 0; t <= kSteps; ++t) {
            sa[t * kWave] = i + t < a ? ra[t] : kPastEnd;
            sb[t * kWave] = j + t < b ? rb[t] : kPastEnd;
          }
        }
        int32_t ia = 0, ib = 0;
        int32_t av = sa[0], bv = sb[0];
        for (int st = 0; st < q; ++st) {
          const bool take_a = av <= bv;
          if (take_a && av == bv) {
            ++cuv;
            if (Support) {
              atomicAdd(&sup[ab + i + ia], 1u);  // the edge (u, w)
              atomicAdd(&sup[bb + j + ib], 1u);  // the edge (v, w)
            }
          }
          // one LDS read per step: the next element of the list just taken from
          if (take_a) ++ia;
          else ++ib;
          const int32_t x = take_a ? sa[ia * kWave] : sb[ib * kWave];
          if (take_a) av = x;
          else bv = x;
        }
        i += ia;
        j += ib;
        p += q;
      }
      hits += cuv;
      if (Support && cuv) atomicAdd(&sup[e], cuv);  // the edge (u, v)
      if (p >= pend) break;
      e = gallop_upper(P, e + 1, e_hi + 2, p) - 1;
    }
  }
  const uint64_t wh = (uint64_t)wave_sum((int64_t)hits);
  if (lane == 0 && wh) atomicAdd((unsigned long long*)total, (unsigned long long)wh);
}

struct IntersectLayout {
  int32_t* src_of;
  uint32_t* work;
  int64_t* P;
  int64_t* partial;
  size_t bytes;
};

IntersectLayout carve_intersect(void* ws, int64_t cap) {
  Carver c(ws);
  IntersectLayout L;
  L.src_of = c.take<int32_t>(cap);
  L.work = c.take<uint32_t>(cap);
  L.P = c.take<int64_t>(cap + 1);
  L.partial = c.take<int64_t>(scan_partial_len(cap));
  L.bytes = c.used();
  return L;
}

template <typename OffT>
tc_status intersect_impl(int64_t n, const OffT* rp, const int32_t* col, int64_t cap,
                         uint64_t* total, uint32_t* sup, int64_t* m_out, const IntersectLayout& L,
                         hipStream_t s) {
  intersect_init_kernel<<<1, 1, 0, s>>>(total);
  edge_work_kernel<OffT><<<grid_for(std::max<int64_t>(n, cap / 64), 256 / kWave, 8192), 256, 0, s>>>(
      n, rp, col, cap, L.src_of, L.work, m_out);
  hipError_t e = scan_exclusive<OpSum>(cap, WorkLoad{L.work}, PrefixStore{L.P}, L.partial, s);
  if (e != hipSuccess) return check_hip(e, "segmented intersection scan");
  intersect_finish_scan_kernel<<<1, 1, 0, s>>>(L.partial, scan_num_tiles(cap), cap, L.P);
  if (sup) clear_u32_kernel<<<grid_for(cap, 256, 8192), 256, 0, s>>>(sup, m_out);
  // 4 workgroups per CU (the launch bound): about 105 VGPRs per lane; bounds of 5 and 6
  // fit the LDS staging too but spill registers and were slower
  const int grid = 4 * device_cu_count();
  const bool narrow = cap < (int64_t(1) << 30);
  if (sup && narrow)
    merge_kernel<true, true, OffT><<<grid, kBlock, 0, s>>>(cap, rp, col, L.src_of, L.P, m_out,
                                                           total, sup);
  else if (sup)
    merge_kernel<true, false, OffT><<<grid, kBlock, 0, s>>>(cap, rp, col, L.src_of, L.P, m_out,
                                                            total, sup);
  else if (narrow)
    merge_kernel<false, true, OffT><<<grid, kBlock, 0, s>>>(cap, rp, col, L.src_of, L.P, m_out,
                                                            total, nullptr);
  else
    merge_kernel<false, false, OffT><<<grid, kBlock, 0, s>>>(cap, rp, col, L.src_of, L.P, m_out,
                                                             total, nullptr);
  return check_hip(hipGetLastError(), "tc_segmented_intersect launch");
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_segmented_intersect(const tc_csr* dag, int64_t edge_capacity,
                                            uint64_t* total, uint32_t* support, int64_t* m_out,
                                            void* ws, size_t* ws_bytes, void* stream) {
  using namespace tc;
  if (!dag) return fail(TC_ERR_INVALID_ARG, "dag is NULL");
  const int64_t n = dag->n;
  if (n < 0) return fail(TC_ERR_INVALID_ARG, "negative n");
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (dag->offset_bytes != 4 && dag->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", dag->offset_bytes);
  if (edge_capacity < 0) return fail(TC_ERR_INVALID_ARG, "negative edge_capacity");
  if (edge_capacity > ((int64_t)1 << 40))
    return fail(TC_ERR_UNSUPPORTED, "edge_capacity=%lld is beyond 2^40", (long long)edge_capacity);
  tc_status st;
  if (workspace_query(ws, ws_bytes, carve_intersect(nullptr, edge_capacity).bytes, &st)) return st;
  if (!dag->row_ptr || !total || !m_out) return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const IntersectLayout L = carve_intersect(ws, edge_capacity);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dag->offset_bytes == 4)
    st = intersect_impl<int32_t>(n, static_cast<const int32_t*>(dag->row_ptr), dag->col,
                                 edge_capacity, total, support, m_out, L, s);
  else
    st = intersect_impl<int64_t>(n, static_cast<const int64_t*>(dag->row_ptr), dag->col,
                                 edge_capacity, total, support, m_out, L, s);
  return st == TC_OK ? ok() : st;
}
