// pack.hip - tc_pack_pairs: the raw pairs of many graphs, concatenated, moved
// to the global ids of their disjoint union.
//
// A batch of graphs is counted as one disjoint union whose graph g owns the
// vertex ids [vtx_off[g], vtx_off[g+1]).  The pairs of graph g arrive with
// local ids at positions [pair_off[g], pair_off[g+1]) of the concatenated
// arrays; this adds vtx_off[g] to both ends of each of them, in place, so the
// union can be cleaned by tc_build_csr in one call.  A local id outside
// [0, vtx_off[g+1] - vtx_off[g]) becomes -1 instead, so it cannot land in
// another graph: tc_build_csr then reports TC_ERR_ID_OUT_OF_RANGE for the
// batch.  One workgroup per graph (grid-stride over the graphs), coalesced over
// its pairs.
#include "tc_device.h"
#include "tc_host.h"

namespace tc {
namespace {

constexpr int kPackBlock = 256;

__global__ __launch_bounds__(kPackBlock) void pack_pairs_kernel(int64_t num_graphs,
                                                                const int64_t* __restrict__ pair_off,
                                                                const int64_t* __restrict__ vtx_off,
                                                                int32_t* __restrict__ src,
                                                                int32_t* __restrict__ dst) {
  for (int64_t g = blockIdx.x; g < num_graphs; g += gridDim.x) {
    const int64_t b = pair_off[g], e = pair_off[g + 1];
    const int64_t shift = vtx_off[g], ng = vtx_off[g + 1] - shift;
    for (int64_t i = b + threadIdx.x; i < e; i += kPackBlock) {
      const int32_t a = src[i], c = dst[i];
      src[i] = a >= 0 && a < ng ? (int32_t)(a + shift) : -1;
      dst[i] = c >= 0 && c < ng ? (int32_t)(c + shift) : -1;
    }
  }
}

}  // namespace
}  // namespace tc

extern "C" tc_status tc_pack_pairs(int64_t num_graphs, const int64_t* pair_off,
                                   const int64_t* vtx_off, int32_t* src, int32_t* dst,
                                   void* stream) {
  using namespace tc;
  if (num_graphs < 0 || num_graphs > INT32_MAX)
    return fail(TC_ERR_INVALID_ARG, "num_graphs=%lld out of range", (long long)num_graphs);
  if (num_graphs == 0) return ok();
  if (!pair_off || !vtx_off || !src || !dst) return fail(TC_ERR_INVALID_ARG, "null device pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = grid_for(num_graphs, 1, 8192);
  pack_pairs_kernel<<<grid, kPackBlock, 0, s>>>(num_graphs, pair_off, vtx_off, src, dst);
  const tc_status st = check_hip(hipGetLastError(), "tc_pack_pairs launch");
  return st == TC_OK ? ok() : st;
}
