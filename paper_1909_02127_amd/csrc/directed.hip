// directed.hip - per-edge codes of the DAG from the input pairs:
// tc_edge_directions (which way each edge points in a directed data graph) and
// tc_edge_labels (each edge's label in an edge-labelled one).
//
// The build and the orientation keep the undirected edges (the method is
// stated for undirected graphs, Sec. II-A, which also says it extends to
// directed ones).  A directed query then needs, for every DAG edge, the arcs
// of the data graph between its two vertices: one byte per edge, aligned with
// the DAG's column array, bit 0 for the arc from the row's vertex to the
// column, bit 1 for the reverse.  One thread per input arc finds its edge by
// binary search of the two rows (the edge is stored in exactly one of them).
#include "tc_device.h"
#include "tc_host.h"

namespace tc {
namespace {

// m_out = m, or -TC_ERR_CAPACITY when m > cap; the direction words of [0, m)
// cleared.
template <typename OffT>
__global__ void dir_clear_kernel(const OffT* __restrict__ rp, int64_t n, int64_t cap,
                                 uint32_t* __restrict__ words, int64_t* __restrict__ m_out) {
  const int64_t m = (int64_t)rp[n];
  if (blockIdx.x == 0 && threadIdx.x == 0) *m_out = m > cap ? -(int64_t)TC_ERR_CAPACITY : m;
  if (m > cap) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (m + 3) / 4; i += stride)
    words[i] = 0u;
}

// Position of x in the ascending row col[beg, end), or -1.
__device__ __forceinline__ int64_t row_find(const int32_t* __restrict__ col, int64_t beg,
                                            int64_t end, int32_t x) {
  int64_t lo = beg, hi = end;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < end && col[lo] == x ? lo : -1;
}

// Every arc s -> d (s != d) sets one bit of the DAG edge between s and d: bit 0
// when the edge is stored in s's row (the arc leaves the row's vertex), bit 1
// when it is stored in d's row.  Bytes are set through their 32-bit words.
template <typename OffT>
__global__ __launch_bounds__(256) void dir_arcs_kernel(const OffT* __restrict__ rp, int64_t n,
                                                       const int32_t* __restrict__ col,
                                                       int64_t num_pairs,
                                                       const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ dst,
                                                       uint32_t* __restrict__ words,
                                                       int64_t* __restrict__ m_out) {
  if (*m_out < 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < num_pairs; i += stride) {
    const int32_t a = src[i], b = dst[i];
    if (a < 0 || a >= n || b < 0 || b >= n) {
      *m_out = -(int64_t)TC_ERR_ID_OUT_OF_RANGE;
      continue;
    }
    if (a == b) continue;
    // the shorter row first: degree orders put an edge in its lower-degree end's row
    const int64_t ab = (int64_t)rp[a], ae = (int64_t)rp[a + 1];
    const int64_t bb = (int64_t)rp[b], be = (int64_t)rp[b + 1];
    const bool a_first = ae - ab <= be - bb;
    int64_t pos = a_first ? row_find(col, ab, ae, b) : row_find(col, bb, be, a);
    uint32_t bit = a_first ? 1u : 2u;
    if (pos < 0) {
      pos = a_first ? row_find(col, bb, be, a) : row_find(col, ab, ae, b);
      bit ^= 3u;
    }
    if (pos < 0) {
      *m_out = -(int64_t)TC_ERR_INVALID_ARG;  // not an edge of this DAG
      continue;
    }
    atomicOr(&words[pos >> 2], bit << ((pos & 3) * 8));
  }
}

tc_status check_edge_dag(const tc_csr* dag, int64_t edge_capacity) {
  if (!dag) return fail(TC_ERR_INVALID_ARG, "dag is NULL");
  if (dag->n < 0) return fail(TC_ERR_INVALID_ARG, "negative n");
  if (dag->n > INT32_MAX)
    return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)dag->n);
  if (dag->offset_bytes != 4 && dag->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", dag->offset_bytes);
  if (edge_capacity < 0) return fail(TC_ERR_INVALID_ARG, "negative edge_capacity");
  if (edge_capacity > ((int64_t)1 << 40))
    return fail(TC_ERR_UNSUPPORTED, "edge_capacity=%lld is beyond 2^40", (long long)edge_capacity);
  return TC_OK;
}

// Every labelled pair {a, b} (a != b) raises the byte of the DAG edge between
// a and b to its label (the largest label of an edge's pairs wins), through a
// compare-and-swap of the byte's 32-bit word; a label above kMaxEdgeLabel is
// reported as -TC_ERR_INVALID_ARG.
constexpr int32_t kMaxEdgeLabel = 3;

template <typename OffT>
__global__ __launch_bounds__(256) void edge_label_kernel(const OffT* __restrict__ rp, int64_t n,
                                                         const int32_t* __restrict__ col,
                                                         int64_t num_pairs,
                                                         const int32_t* __restrict__ src,
                                                         const int32_t* __restrict__ dst,
                                                         const uint8_t* __restrict__ labels,
                                                         uint32_t* __restrict__ words,
                                                         int64_t* __restrict__ m_out) {
  if (*m_out < 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < num_pairs; i += stride) {
    const int32_t a = src[i], b = dst[i];
    if (a < 0 || a >= n || b < 0 || b >= n) {
      *m_out = -(int64_t)TC_ERR_ID_OUT_OF_RANGE;
      continue;
    }
    if (a == b) continue;
    const uint32_t lab = labels[i];
    if (lab > (uint32_t)kMaxEdgeLabel) {
      *m_out = -(int64_t)TC_ERR_INVALID_ARG;
      continue;
    }
    // the shorter row first: degree orders put an edge in its lower-degree end's row
    const int64_t ab = (int64_t)rp[a], ae = (int64_t)rp[a + 1];
    const int64_t bb = (int64_t)rp[b], be = (int64_t)rp[b + 1];
    const bool a_first = ae - ab <= be - bb;
    int64_t pos = a_first ? row_find(col, ab, ae, b) : row_find(col, bb, be, a);
    if (pos < 0) pos = a_first ? row_find(col, bb, be, a) : row_find(col, ab, ae, b);
    if (pos < 0) {
      *m_out = -(int64_t)TC_ERR_INVALID_ARG;  // not an edge of this DAG
      continue;
    }
    uint32_t* w = &words[pos >> 2];
    const int sh = (int)(pos & 3) * 8;
    uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (((old >> sh) & 0xFFu) < lab) {
      const uint32_t want = (old & ~(0xFFu << sh)) | (lab << sh);
      const uint32_t seen = atomicCAS(w, old, want);
      if (seen == old) break;
      old = seen;
    }
  }
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_edge_labels(const tc_csr* dag, int64_t edge_capacity, int64_t num_pairs,
                                    const int32_t* src, const int32_t* dst, const uint8_t* labels,
                                    uint8_t* edge_labels, int64_t* m_out, void* stream) {
  using namespace tc;
  tc_status st = check_edge_dag(dag, edge_capacity);
  if (st != TC_OK) return st;
  if (num_pairs < 0) return fail(TC_ERR_INVALID_ARG, "negative num_pairs");
  if (!dag->row_ptr || !m_out || (edge_capacity > 0 && !edge_labels) ||
      (num_pairs > 0 && (!src || !dst || !labels)))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(edge_labels) % 4 != 0)
    return fail(TC_ERR_INVALID_ARG, "edge_labels must be 4-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* words = reinterpret_cast<uint32_t*>(edge_labels);
  const int cg = grid_for((edge_capacity + 3) / 4, 256, 8192);
  const int ag = grid_for(num_pairs, 256, 16384);
  if (dag->offset_bytes == 4) {
    const int32_t* rp = static_cast<const int32_t*>(dag->row_ptr);
    dir_clear_kernel<int32_t><<<cg, 256, 0, s>>>(rp, dag->n, edge_capacity, words, m_out);
    if (num_pairs > 0)
      edge_label_kernel<int32_t><<<ag, 256, 0, s>>>(rp, dag->n, dag->col, num_pairs, src, dst,
                                                    labels, words, m_out);
  } else {
    const int64_t* rp = static_cast<const int64_t*>(dag->row_ptr);
    dir_clear_kernel<int64_t><<<cg, 256, 0, s>>>(rp, dag->n, edge_capacity, words, m_out);
    if (num_pairs > 0)
      edge_label_kernel<int64_t><<<ag, 256, 0, s>>>(rp, dag->n, dag->col, num_pairs, src, dst,
                                                    labels, words, m_out);
  }
  return check_hip(hipGetLastError(), "tc_edge_labels launch") == TC_OK ? ok() : TC_ERR_HIP;
}

extern "C" tc_status tc_edge_directions(const tc_csr* dag, int64_t edge_capacity,
                                        int64_t num_pairs, const int32_t* src,
                                        const int32_t* dst, uint8_t* dir, int64_t* m_out,
                                        void* stream) {
  using namespace tc;
  tc_status st = check_edge_dag(dag, edge_capacity);
  if (st != TC_OK) return st;
  if (num_pairs < 0) return fail(TC_ERR_INVALID_ARG, "negative num_pairs");
  if (!dag->row_ptr || !m_out || (edge_capacity > 0 && !dir) || (num_pairs > 0 && (!src || !dst)))
    return fail(TC_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(dir) % 4 != 0)
    return fail(TC_ERR_INVALID_ARG, "dir must be 4-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* words = reinterpret_cast<uint32_t*>(dir);
  const int cg = grid_for((edge_capacity + 3) / 4, 256, 8192);
  const int ag = grid_for(num_pairs, 256, 16384);
  if (dag->offset_bytes == 4) {
    const int32_t* rp = static_cast<const int32_t*>(dag->row_ptr);
    dir_clear_kernel<int32_t><<<cg, 256, 0, s>>>(rp, dag->n, edge_capacity, words, m_out);
    if (num_pairs > 0)
      dir_arcs_kernel<int32_t><<<ag, 256, 0, s>>>(rp, dag->n, dag->col, num_pairs, src, dst, words,
                                                  m_out);
  } else {
    const int64_t* rp = static_cast<const int64_t*>(dag->row_ptr);
    dir_clear_kernel<int64_t><<<cg, 256, 0, s>>>(rp, dag->n, edge_capacity, words, m_out);
    if (num_pairs > 0)
      dir_arcs_kernel<int64_t><<<ag, 256, 0, s>>>(rp, dag->n, dag->col, num_pairs, src, dst, words,
                                                  m_out);
  }
  return check_hip(hipGetLastError(), "tc_edge_directions launch") == TC_OK ? ok() : TC_ERR_HIP;
}

