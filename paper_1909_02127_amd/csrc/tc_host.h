// tc_host.h - host-side helpers shared by the C ABI entry points of libtc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tc.h"

namespace tc {

// Records a thread-local message for tc_last_error() and returns `status`.
tc_status fail(tc_status status, const char* fmt, ...);
// Clears the thread-local message and returns TC_OK.
tc_status ok();

// Maps a HIP error from a launch or runtime call to TC_ERR_HIP (with message).
tc_status check_hip(hipError_t err, const char* what);

// Compute units and the registered-kernel occupancy of the current device.
int device_cu_count();

// Sequential carving of one caller-provided workspace into 256-byte-aligned
// regions.  With base == nullptr it only measures.
class Carver {
 public:
  explicit Carver(void* base) : base_(static_cast<char*>(base)) {}
  template <typename T>
  T* take(int64_t count) {
    size_t bytes = (size_t)(count > 0 ? count : 0) * sizeof(T);
    size_t at = used_;
    used_ = align(used_ + bytes);
    return base_ ? reinterpret_cast<T*>(base_ + at) : nullptr;
  }
  size_t used() const { return used_ == 0 ? 256 : used_; }

 private:
  static size_t align(size_t x) { return (x + 255) & ~(size_t)255; }
  char* base_;
  size_t used_ = 0;
};

// Workspace protocol: query (ws == NULL) or check the caller's size.
// Returns true when the caller only asked for the size (already written).
bool workspace_query(void* ws, size_t* ws_bytes, size_t need, tc_status* status);

// The count kernel's coded launch for a triangle query with edge labels q (each
// 0..3): every closed wedge adds the query's matches on its triangle, by the
// labels of its three edges (count.hip); workspace protocol as tc_count's.
tc_status count_coded_edge_labels(const tc_csr* dag, const uint8_t* edge_labels, const int32_t q[3],
                                  uint64_t* total, const tc_tune* tune, void* ws,
                                  size_t* ws_bytes, void* stream);

inline int grid_for(int64_t work, int block, int cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace tc
