// work.hip - tc_source_work: the wedge work of every source and its prefix.
//
// In the all-source advance (Alg. 1 "Advance", Sec. III-B) source u enumerates
// one wedge u -> v -> w for every v in N+(u) and w in N+(v), so its work is
// w(u) = sum of d+(v) over its middles; a source with d+(u) < 2 closes no wedge
// and is not advanced (the 2-look-ahead of Sec. III-C), so its work is 0.  The
// exclusive prefix of w over the vertex ids splits the sources into ranges of
// equal work: the cut a shard planner takes, and the total W that sizes the
// count's memory traffic.
#include "tc_device.h"
#include "tc_host.h"
#include "tc_scan.h"

#include <algorithm>

namespace tc {
namespace {

// w(u) for every vertex: one wave per source, the middles' out-degrees summed
// over the wave.
template <typename OffT>
__global__ __launch_bounds__(256) void source_work_kernel(int64_t n, const OffT* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          int64_t* __restrict__ work) {
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; u < n;
       u += nwaves) {
    const int64_t beg = (int64_t)rp[u];
    const int64_t d = (int64_t)rp[u + 1] - beg;
    int64_t w = 0;
    if (d >= 2) {
      for (int64_t i = lane; i < d; i += kWave) {
        const int32_t v = col[beg + i];
        w += (int64_t)rp[v + 1] - (int64_t)rp[v];
      }
      w = wave_sum(w);
    }
    if (lane == 0) work[u] = w;
  }
}

struct WorkLoad {
  const int64_t* work;
  __device__ int64_t operator()(int64_t i) const { return work[i]; }
};
struct PrefixStore {
  int64_t* p;
  __device__ void operator()(int64_t i, int64_t x) const { p[i] = x; }
};

__global__ void work_total_kernel(const int64_t* __restrict__ partial, int64_t tiles, int64_t n,
                                  int64_t* __restrict__ prefix) {
  prefix[n] = tiles > 0 ? partial[tiles] : 0;
}

struct WorkLayout {
  int64_t* work;  // used when the caller passes no work array
  int64_t* partial;
  size_t bytes;
};

WorkLayout carve_work(void* ws, int64_t n) {
  Carver c(ws);
  WorkLayout L;
  L.work = c.take<int64_t>(n);
  L.partial = c.take<int64_t>(scan_partial_len(n));
  L.bytes = c.used();
  return L;
}

template <typename OffT>
tc_status work_impl(int64_t n, const OffT* rp, const int32_t* col, int64_t* work, int64_t* prefix,
                    const WorkLayout& L, hipStream_t s) {
  if (n > 0)
    source_work_kernel<OffT><<<grid_for(n, 256 / kWave, 16384), 256, 0, s>>>(n, rp, col, work);
  hipError_t e = scan_exclusive<OpSum>(n, WorkLoad{work}, PrefixStore{prefix}, L.partial, s);
  if (e != hipSuccess) return check_hip(e, "source work scan");
  work_total_kernel<<<1, 1, 0, s>>>(L.partial, scan_num_tiles(n), n, prefix);
  return check_hip(hipGetLastError(), "tc_source_work launch");
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_source_work(const tc_csr* dag, int64_t* work, int64_t* prefix, void* ws,
                                    size_t* ws_bytes, void* stream) {
  using namespace tc;
  if (!dag) return fail(TC_ERR_INVALID_ARG, "dag is NULL");
  const int64_t n = dag->n;
  if (n < 0) return fail(TC_ERR_INVALID_ARG, "negative n");
  if (n > INT32_MAX) return fail(TC_ERR_UNSUPPORTED, "n=%lld needs ids beyond int32", (long long)n);
  if (dag->offset_bytes != 4 && dag->offset_bytes != 8)
    return fail(TC_ERR_INVALID_ARG, "offset_bytes must be 4 or 8, got %d", dag->offset_bytes);
  tc_status st;
  if (workspace_query(ws, ws_bytes, carve_work(nullptr, n).bytes, &st)) return st;
  if (!dag->row_ptr || !prefix) return fail(TC_ERR_INVALID_ARG, "null device pointer");
  const WorkLayout L = carve_work(ws, n);
  int64_t* w = work ? work : L.work;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dag->offset_bytes == 4)
    st = work_impl<int32_t>(n, static_cast<const int32_t*>(dag->row_ptr), dag->col, w, prefix, L, s);
  else
    st = work_impl<int64_t>(n, static_cast<const int64_t*>(dag->row_ptr), dag->col, w, prefix, L, s);
  return st == TC_OK ? ok() : st;
}
