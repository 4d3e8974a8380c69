// label.hip - tc_count_labelled: triangles whose vertex labels match a
// labelled triangle query.
//
// A match of a labelled query must map every query node to a data vertex of the
// same label (Sec. I: structure and node labels are matched; Sec. II-A: the
// method extends to queries with node labels).  Alg. 1 starts by filtering the
// candidate set (Filter+Compute); with labels, a data edge (u, v) can match a
// query edge only when the pair of labels {L(u), L(v)} is one of the query's
// three edge label pairs, i.e. a sub-multiset of the query labels {a, b, c}.
// The filter keeps exactly those oriented edges, compacted into a DAG of the
// same vertex set, and the count then runs unchanged on it:
//   - a triangle of the filtered graph has all three edges kept; for a query
//     with three equal or three distinct labels that already forces its label
//     multiset to be the query's, so its count is the answer;
//   - for {a, a, b} (a != b) the filtered graph also keeps the triangles of
//     {a, a, a} (every edge is {a, a}), so the count of {a, a, a}, filtered
//     and counted the same way, is subtracted.
// In the neighbourhood-equivalence terms of Def. 3, the query's classes are its
// groups of equal labels; the orientation of the DAG orders the members of
// each class, and vertices of distinct labels are told apart by the labels, so
// every labelled match is counted once.
#include "tc_device.h"
#include "tc_host.h"
#include "tc_scan.h"

#include <algorithm>

namespace tc {
namespace {

// The query labels in ascending order.
struct Query {
  int32_t q0, q1, q2;
};

__device__ __forceinline__ bool label_in(const Query& q, int32_t x) {
  return x == q.q0 || x == q.q1 || x == q.q2;
}

// {x, y} is a sub-multiset of {q0, q1, q2}: the sorted pair equals the query
// with one label removed.
__device__ __forceinline__ bool pair_fits(const Query& q, int32_t x, int32_t y) {
  const int32_t lo = x < y ? x : y;
  const int32_t hi = x < y ? y : x;
  return (lo == q.q0 && (hi == q.q1 || hi == q.q2)) || (lo == q.q1 && hi == q.q2);
}

// One wave takes kRows consecutive rows at a time and walks their edges as one
// contiguous range of the column array, 64 edges per step, the loads of
// kSteps steps in flight together.  A lane finds its edge's row as the
// short-list walk of the count does: every non-empty row marks its first
// position of the step in LDS with (row << 6 | position), and a wave max-scan
// hands each lane the last row that starts at or before it (and where that
// row's part of the step begins).  The last lane of a row's part adds the
// row's kept edges of the step from the ballot to the row's LDS counter.
constexpr int kRows = 32;
constexpr int kSteps = 4;
static_assert(kRows < kWave, "row bounds are held one per lane");
constexpr int32_t kNoMark = -1;

// Lanes [lo, hi) of a 64-lane mask (0 <= lo <= hi <= 64).
__device__ __forceinline__ uint64_t lane_range(int lo, int hi) {
  const uint64_t upto_hi = hi >= kWave ? ~uint64_t(0) : (uint64_t(1) << hi) - 1;
  const uint64_t upto_lo = (uint64_t(1) << lo) - 1;
  return hi > lo ? upto_hi & ~upto_lo : 0;
}

// Per-wave LDS of the walk.
struct WalkLds {
  int32_t mark[kWave];   // kNoMark between steps
  int32_t count[kRows];  // per row: kept edges (pass 1), edges written (pass 2)
  int64_t at[kRows];     // pass 2: the rows' new offsets
};

// Rows and part starts of the steps s0 = e0 + k 64 (k < kSteps) of the edge
// range [e_beg, e_end) whose rows start at bnd (lane r < kRows: row r's first
// edge; nonempty: row r has an edge).  carry: the packed row of the last lane
// of the previous step (its part continues at position 0), updated.
__device__ __forceinline__ void walk_rows(WalkLds& L, int64_t bnd, bool nonempty, int64_t e0,
                                          int64_t e_end, int32_t& carry, int32_t (&row)[kSteps],
                                          int32_t (&seg0)[kSteps]) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < kSteps; ++k) {
    const int64_t s0 = e0 + k * kWave;
    row[k] = 0;
    seg0[k] = 0;
    if (s0 >= e_end) continue;  // uniform
    const int64_t rel = bnd - s0;
    const bool marks = nonempty && rel >= 0 && rel < kWave;
    if (marks) L.mark[rel] = (lane << 6) | (int32_t)rel;
    wave_sync();
    int32_t pk = wave_inclusive_max32(L.mark[lane]);
    pk = pk > carry ? pk : carry;
    wave_sync();
    if (marks) L.mark[rel] = kNoMark;
    carry = read_lane(pk, kWave - 1) & ~63;  // the same row, from position 0 of the next step
    row[k] = pk >> 6;
    seg0[k] = pk & 63;
  }
}

// Reports whether the DAG fits the caller's edge capacity; every later kernel
// reads this status and does nothing (or writes an empty DAG) when it fails.
template <typename OffT>
__global__ void label_status_kernel(const OffT* __restrict__ rp, int64_t n, int64_t cap,
                                    int64_t* __restrict__ status, uint64_t* __restrict__ totals) {
  const int64_t m = (int64_t)rp[n];
  *status = m > cap ? -(int64_t)TC_ERR_CAPACITY : m;
  totals[0] = 0;
  totals[1] = 0;
}

// Pass 1: kept out-degree of every source, and the keep flag of each edge it
// reads.  Node labels (Edge false): the edges of the sources whose label is in
// the query (the rows of the others are not read and keep nothing), kept when
// the pair of labels fits the query.  Edge labels (Edge true): every edge,
// kept when its own label is one of the query's.
template <typename OffT, bool Edge>
__global__ __launch_bounds__(256) void label_degree_kernel(
    int64_t n, const OffT* __restrict__ rp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ labels, const uint8_t* __restrict__ elab, Query q,
    const int64_t* __restrict__ status, uint8_t* __restrict__ keep, int64_t* __restrict__ deg) {
  __shared__ WalkLds lds_all[256 / kWave];
  WalkLds& L = lds_all[threadIdx.x / kWave];
  const int lane = lane_id();
  L.mark[lane] = kNoMark;
  wave_sync();
  const bool bad = *status < 0;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kWave) * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kRows;
       r0 < n; r0 += stride) {
    // lanes 0..kRows: the rows' bounds (clamped at n); lanes < kRows: the rows' labels
    const int64_t x = r0 + lane < n ? r0 + lane : n;
    const int64_t bnd = lane <= kRows ? (int64_t)rp[x] : 0;
    const bool row_ok = lane < kRows && r0 + lane < n;
    const int32_t lab = !Edge && row_ok ? labels[r0 + lane] : 0;
    const uint64_t cand = ballot(row_ok && !bad && (Edge || label_in(q, lab)));
    // cross-lane reads are made by every lane, outside any condition (a lane
    // reading from one that skipped the instruction would get no value)
    const int64_t bnd_next = __shfl_down(bnd, 1, kWave);
    const bool nonempty = row_ok && bnd_next > bnd;
    const int64_t e_beg = read_lane64(bnd, 0), e_end = read_lane64(bnd, kRows);
    if (lane < kRows) L.count[lane] = 0;
    wave_sync();
    int32_t carry = kNoMark;
    for (int64_t e0 = e_beg; cand && e0 < e_end; e0 += kSteps * kWave) {
      int32_t row[kSteps], seg0[kSteps], v[kSteps], lv[kSteps];
      bool act[kSteps];
      walk_rows(L, bnd, nonempty, e0, e_end, carry, row, seg0);
#pragma unroll
      for (int k = 0; k < kSteps; ++k) {
        const int64_t e = e0 + k * kWave + lane;
        act[k] = e < e_end && ((cand >> row[k]) & 1);
        // edge labels: the edge's own label; node labels: the column, then its label
        v[k] = act[k] ? (Edge ? (int32_t)elab[e] : col[e]) : 0;
      }
#pragma unroll
      for (int k = 0; k < kSteps; ++k) lv[k] = !Edge && act[k] ? labels[v[k]] : 0;
#pragma unroll
      for (int k = 0; k < kSteps; ++k) {
        const int64_t e = e0 + k * kWave + lane;
        const int32_t lu = __shfl(lab, row[k], kWave);
        const bool kp = act[k] && (Edge ? label_in(q, v[k]) : pair_fits(q, lu, lv[k]));
        if (act[k]) keep[e] = (uint8_t)kp;
        const uint64_t b = ballot(kp);
        // the last lane of each row's part of the step adds the part's kept edges
        const bool in = e < e_end;
        const int32_t row_next = __shfl_down(row[k], 1, kWave);
        const bool next_same = lane + 1 < kWave && e + 1 < e_end && row_next == row[k];
        if (in && !next_same) L.count[row[k]] += (int32_t)popc(b & lane_range(seg0[k], lane + 1));
        wave_sync();
      }
    }
    if (row_ok) deg[r0 + lane] = L.count[lane];
    wave_sync();
  }
}

struct DegLoad {
  const int64_t* deg;
  __device__ int64_t operator()(int64_t i) const { return deg[i]; }
};
struct OffStore {
  int64_t* off;
  __device__ void operator()(int64_t i, int64_t x) const { off[i] = x; }
};

// Pass 2: the kept edges of every row, in their order, at the row's new
// offset; the new row offsets.  Only rows that keep something are read (their
// keep flags were written by pass 1).  When the capacity check failed, or the
// kept edges exceed the capacity, every row is written empty (the count then
// sees a graph with no edges).
template <typename OffT, bool Edge>
__global__ __launch_bounds__(256) void label_compact_kernel(
    int64_t n, const OffT* __restrict__ rp, const int32_t* __restrict__ col,
    const uint8_t* __restrict__ keep, const int64_t* __restrict__ off,
    const int64_t* __restrict__ partial, int64_t tiles, int64_t cap,
    const int64_t* __restrict__ status, OffT* __restrict__ frp, int32_t* __restrict__ fcol,
    const uint8_t* __restrict__ elab, uint8_t* __restrict__ flab) {
  __shared__ WalkLds lds_all[256 / kWave];
  WalkLds& L = lds_all[threadIdx.x / kWave];
  const int lane = lane_id();
  L.mark[lane] = kNoMark;
  wave_sync();
  const int64_t kept_total = tiles > 0 ? partial[tiles] : 0;
  const bool empty = *status < 0 || kept_total > cap;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kWave) * kRows;
  int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kRows;
  if (r0 == 0 && lane == 0) frp[n] = (OffT)(empty ? 0 : kept_total);
  for (; r0 < n; r0 += stride) {
    const int64_t x = r0 + lane < n ? r0 + lane : n;
    const int64_t bnd = lane <= kRows ? (int64_t)rp[x] : 0;
    const bool row_ok = lane < kRows && r0 + lane < n;
    // lanes 0..kRows: the rows' new offsets (the one past the last row: the next row's)
    const int64_t at = lane <= kRows && !empty ? (x < n ? off[x] : kept_total) : 0;
    if (row_ok) frp[r0 + lane] = (OffT)at;
    const int64_t at_next = __shfl_down(at, 1, kWave);
    const uint64_t rows = ballot(row_ok && at_next > at);  // rows that keep something
    // cross-lane reads are made by every lane, outside any condition (a lane
    // reading from one that skipped the instruction would get no value)
    const int64_t bnd_next = __shfl_down(bnd, 1, kWave);
    const bool nonempty = row_ok && bnd_next > bnd;
    const int64_t e_beg = read_lane64(bnd, 0), e_end = read_lane64(bnd, kRows);
    if (lane < kRows) {
      L.count[lane] = 0;
      L.at[lane] = at;
    }
    wave_sync();
    int32_t carry = kNoMark;
    for (int64_t e0 = e_beg; rows && e0 < e_end; e0 += kSteps * kWave) {
      int32_t row[kSteps], seg0[kSteps], v[kSteps];
      bool kp[kSteps];
      walk_rows(L, bnd, nonempty, e0, e_end, carry, row, seg0);
#pragma unroll
      for (int k = 0; k < kSteps; ++k) {
        const int64_t e = e0 + k * kWave + lane;
        kp[k] = e < e_end && ((rows >> row[k]) & 1) && keep[e];
      }
#pragma unroll
      for (int k = 0; k < kSteps; ++k) v[k] = kp[k] ? col[e0 + k * kWave + lane] : 0;
#pragma unroll
      for (int k = 0; k < kSteps; ++k) {
        const int64_t e = e0 + k * kWave + lane;
        const uint64_t b = ballot(kp[k]);
        // rank in the row: the row's kept edges of earlier steps, then this part's
        if (kp[k]) {
          const int64_t pos = L.at[row[k]] + L.count[row[k]] + popc(b & lane_range(seg0[k], lane));
          fcol[pos] = v[k];
          if (Edge) flab[pos] = elab[e];  // the kept edge's label moves with it
        }
        const bool in = e < e_end;
        const int32_t row_next = __shfl_down(row[k], 1, kWave);
        const bool next_same = lane + 1 < kWave && e + 1 < e_end && row_next == row[k];
        wave_sync();
        if (in && !next_same) L.count[row[k]] += (int32_t)popc(b & lane_range(seg0[k], lane + 1));
        wave_sync();
      }
    }
  }
}

// total = t[0] - t[1] (the second count is 0 unless the query is {a, a, b}),
// 0 on a capacity error; kept_out = the filtered edges of the query, or the
// error.
__global__ void label_finish_kernel(const uint64_t* __restrict__ t,
                                    const int64_t* __restrict__ status, const int64_t* __restrict__ partial,
                                    int64_t tiles, int64_t cap, uint64_t* __restrict__ total,
                                    int64_t* __restrict__ kept_out) {
  const int64_t kept = tiles > 0 ? partial[tiles] : 0;
  const bool err = *status < 0 || kept > cap;
  *total = err ? 0 : t[0] - t[1];
  if (kept_out) *kept_out = *status < 0 ? *status : (kept > cap ? -(int64_t)TC_ERR_CAPACITY : kept);
}

struct LabelLayout {
  int64_t* status;
  uint64_t* t;       // the two counts
  uint8_t* keep;     // per-edge flag
  int64_t* deg;      // kept out-degrees
  int64_t* off;      // their exclusive prefix
  int64_t* partial;  // scan partials (the last one is the kept total)
  int64_t* partial2;
  void* frp;         // filtered DAG row offsets (the input's offset type)
  int32_t* fcol;     // filtered DAG columns
  uint8_t* flab;     // edge labels: the kept edges' labels, aligned with fcol
  void* cws;         // tc_count workspace
  size_t cws_bytes;
  size_t bytes;
};

LabelLayout carve_label(void* ws, int64_t n, int64_t cap, int offset_bytes, size_t count_bytes,
                        bool edge = false) {
  Carver c(ws);
  LabelLayout L;
  L.status = c.take<int64_t>(1);
  L.t = c.take<uint64_t>(2);
  L.keep = c.take<uint8_t>(cap);
  L.deg = c.take<int64_t>(n);
  L.off = c.take<int64_t>(n);
  L.partial = c.take<int64_t>(scan_partial_len(n));
  L.partial2 = c.take<int64_t>(scan_partial_len(n));
  L.frp = c.take<char>((n + 1) * offset_bytes);
  L.fcol = c.take<int32_t>(cap);
  L.flab = edge ? c.take<uint8_t>(cap) : nullptr;
  L.cws = c.take<char>((int64_t)count_bytes);
  L.cws_bytes = count_bytes;
  L.bytes = c.used();
  return L;
}

// One filter of the DAG into the compacted DAG (frp, fcol, and with edge labels
// flab).  `partial` receives the scan partials (its last entry is the number of
// kept edges).
template <typename OffT, bool Edge>
tc_status run_filter(const tc_csr* dag, const int32_t* labels, const uint8_t* elab, const Query& q,
                     int64_t cap, const LabelLayout& L, int64_t* partial, hipStream_t s) {
  const int64_t n = dag->n;
  const OffT* rp = static_cast<const OffT*>(dag->row_ptr);
  OffT* frp = static_cast<OffT*>(L.frp);
  // persistent: every wave resident at once (8 workgroups of 4 waves per CU), each
  // taking many row groups
  const int waves_per_block = 256 / kWave;
  const int grid = grid_for((n + kRows - 1) / kRows, waves_per_block, 8 * device_cu_count());
  if (n > 0)
    label_degree_kernel<OffT, Edge><<<grid, 256, 0, s>>>(n, rp, dag->col, labels, elab, q,
                                                         L.status, L.keep, L.deg);
  hipError_t e = scan_exclusive<OpSum>(n, DegLoad{L.deg}, OffStore{L.off}, partial, s);
  if (e != hipSuccess) return check_hip(e, "label filter scan");
  const int64_t tiles = scan_num_tiles(n);
  label_compact_kernel<OffT, Edge><<<n > 0 ? grid : 1, 256, 0, s>>>(
      n, rp, dag->col, L.keep, L.off, partial, tiles, cap, L.status, frp, L.fcol, elab, L.flab);
  return check_hip(hipGetLastError(), "label filter launch");
}

// One filter of the DAG by the query's label pairs, then one count of the
// filtered DAG into *t.
template <typename OffT>
tc_status filter_and_count(const tc_csr* dag, const int32_t* labels, const Query& q, int64_t cap,
                           const LabelLayout& L, int64_t* partial, uint64_t* t,
                           const tc_tune* tune, hipStream_t s) {
  tc_status st = run_filter<OffT, false>(dag, labels, nullptr, q, cap, L, partial, s);
  if (st != TC_OK) return st;
  tc_csr f{dag->n, dag->offset_bytes, L.frp, L.fcol};
  size_t bytes = L.cws_bytes;
  return tc_count(&f, t, tune, L.cws, &bytes, s);
}

// Shared checks of the two labelled entry points.
tc_status check_labelled(const tc_csr* dag, int64_t edge_capacity) {
  if (!dag) return fail(TC_ERR_INVALID_ARG, "dag is NULL");
  const int64_t n = dag->n;
  if (n < 0) return fail(TC_ERR_INVALID_ARG, "negative n");
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (dag->offset_bytes != 4 && dag->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", dag->offset_bytes);
  if (edge_capacity < 0) return fail(TC_ERR_INVALID_ARG, "negative edge_capacity");
  if (edge_capacity > ((int64_t)1 << 40))
    return fail(TC_ERR_UNSUPPORTED, "edge_capacity=%lld is beyond 2^40", (long long)edge_capacity);
  if (dag->offset_bytes == 4 && edge_capacity > INT32_MAX)
    return fail(TC_ERR_INVALID_ARG, "edge_capacity=%lld does not fit 4-byte offsets",
                (long long)edge_capacity);
  return TC_OK;
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_count_labelled(const tc_csr* dag, int64_t edge_capacity,
                                       const int32_t* labels, int32_t a, int32_t b, int32_t c,
                                       uint64_t* total, int64_t* kept_out, const tc_tune* tune,
                                       void* ws, size_t* ws_bytes, void* stream) {
  using namespace tc;
  tc_status st = check_labelled(dag, edge_capacity);
  if (st != TC_OK) return st;
  const int64_t n = dag->n;
  // the count's workspace (also validates the tune)
  size_t count_bytes = 0;
  tc_csr probe{n, dag->offset_bytes, nullptr, nullptr};
  st = tc_count(&probe, nullptr, tune, nullptr, &count_bytes, nullptr);
  if (st != TC_OK) return st;
  const LabelLayout need = carve_label(nullptr, n, edge_capacity, dag->offset_bytes, count_bytes);
  if (workspace_query(ws, ws_bytes, need.bytes, &st)) return st;
  if (!dag->row_ptr || !total || (n > 0 && !labels))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const LabelLayout L = carve_label(ws, n, edge_capacity, dag->offset_bytes, count_bytes);
  int32_t x[3] = {a, b, c};
  std::sort(x, x + 3);
  const Query q{x[0], x[1], x[2]};
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool two_classes = (x[0] == x[1]) != (x[1] == x[2]);  // {a, a, b} or {a, b, b}
  const int32_t twice = x[0] == x[1] ? x[0] : x[2];            // the label that appears twice
  const Query q_same{twice, twice, twice};
  const bool w4 = dag->offset_bytes == 4;
  if (w4)
    label_status_kernel<int32_t><<<1, 1, 0, s>>>(static_cast<const int32_t*>(dag->row_ptr), n,
                                                 edge_capacity, L.status, L.t);
  else
    label_status_kernel<int64_t><<<1, 1, 0, s>>>(static_cast<const int64_t*>(dag->row_ptr), n,
                                                 edge_capacity, L.status, L.t);
  st = w4 ? filter_and_count<int32_t>(dag, labels, q, edge_capacity, L, L.partial, &L.t[0], tune, s)
          : filter_and_count<int64_t>(dag, labels, q, edge_capacity, L, L.partial, &L.t[0], tune, s);
  if (st != TC_OK) return st;
  if (two_classes) {
    st = w4 ? filter_and_count<int32_t>(dag, labels, q_same, edge_capacity, L, L.partial2, &L.t[1],
                                        tune, s)
            : filter_and_count<int64_t>(dag, labels, q_same, edge_capacity, L, L.partial2, &L.t[1],
                                        tune, s);
    if (st != TC_OK) return st;
  }
  label_finish_kernel<<<1, 1, 0, s>>>(L.t, L.status, L.partial, scan_num_tiles(n), edge_capacity,
                                      total, kept_out);
  return check_hip(hipGetLastError(), "tc_count_labelled launch") == TC_OK ? ok() : TC_ERR_HIP;
}

extern "C" tc_status tc_count_edge_labelled(const tc_csr* dag, int64_t edge_capacity,
                                            const uint8_t* edge_labels, int32_t q01, int32_t q02,
                                            int32_t q12, uint64_t* total, int64_t* kept_out,
                                            const tc_tune* tune, void* ws, size_t* ws_bytes,
                                            void* stream) {
  using namespace tc;
  tc_status st = check_labelled(dag, edge_capacity);
  if (st != TC_OK) return st;
  const int64_t n = dag->n;
  int32_t x[3] = {q01, q02, q12};
  // a triangle's three edges are permuted by the permutations of its nodes, so the
  // query is its multiset of edge labels
  std::sort(x, x + 3);
  // the coded count's workspace (also validates the labels and the tune)
  size_t count_bytes = 0;
  tc_csr probe{n, dag->offset_bytes, nullptr, nullptr};
  st = count_coded_edge_labels(&probe, nullptr, x, nullptr, tune, nullptr, &count_bytes, nullptr);
  if (st != TC_OK) return st;
  const LabelLayout need =
      carve_label(nullptr, n, edge_capacity, dag->offset_bytes, count_bytes, true);
  if (workspace_query(ws, ws_bytes, need.bytes, &st)) return st;
  if (!dag->row_ptr || !total || (edge_capacity > 0 && !edge_labels))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const LabelLayout L = carve_label(ws, n, edge_capacity, dag->offset_bytes, count_bytes, true);
  const Query q{x[0], x[1], x[2]};
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool w4 = dag->offset_bytes == 4;
  if (w4)
    label_status_kernel<int32_t><<<1, 1, 0, s>>>(static_cast<const int32_t*>(dag->row_ptr), n,
                                                 edge_capacity, L.status, L.t);
  else
    label_status_kernel<int64_t><<<1, 1, 0, s>>>(static_cast<const int64_t*>(dag->row_ptr), n,
                                                 edge_capacity, L.status, L.t);
  // the edges whose label is one of the query's, then the coded count of those
  st = w4 ? run_filter<int32_t, true>(dag, nullptr, edge_labels, q, edge_capacity, L, L.partial, s)
          : run_filter<int64_t, true>(dag, nullptr, edge_labels, q, edge_capacity, L, L.partial, s);
  if (st != TC_OK) return st;
  tc_csr f{n, dag->offset_bytes, L.frp, L.fcol};
  size_t bytes = L.cws_bytes;
  st = count_coded_edge_labels(&f, L.flab, x, &L.t[0], tune, L.cws, &bytes, s);
  if (st != TC_OK) return st;
  label_finish_kernel<<<1, 1, 0, s>>>(L.t, L.status, L.partial, scan_num_tiles(n), edge_capacity,
                                      total, kept_out);
  return check_hip(hipGetLastError(), "tc_count_edge_labelled launch") == TC_OK ? ok() : TC_ERR_HIP;
}
