// api.cpp - status strings, thread-local error messages and device queries for libtc.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "tc_host.h"

namespace tc {

static thread_local char g_last_error[512] = "";

tc_status fail(tc_status status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return status;
}

tc_status ok() {
  g_last_error[0] = '\0';
  return TC_OK;
}

tc_status check_hip(hipError_t err, const char* what) {
  if (err == hipSuccess) return TC_OK;
  return fail(TC_ERR_HIP, "%s: %s", what, hipGetErrorString(err));
}

int device_cu_count() {
  static std::mutex mu;
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if (cached[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0) {
      cus = 256;
    }
    cached[dev] = cus;
  }
  return cached[dev];
}

bool workspace_query(void* ws, size_t* ws_bytes, size_t need, tc_status* status) {
  if (ws_bytes == nullptr) {
    *status = fail(TC_ERR_INVALID_ARG, "ws_bytes is NULL");
    return true;
  }
  if (ws == nullptr) {
    *ws_bytes = need;
    *status = ok();
    return true;
  }
  if (*ws_bytes < need) {
    *status = fail(TC_ERR_WORKSPACE, "workspace of %zu bytes is below the required %zu", *ws_bytes,
                   need);
    return true;
  }
  if (((uintptr_t)ws & 255u) != 0) {
    *status = fail(TC_ERR_INVALID_ARG, "workspace is not 256-byte aligned");
    return true;
  }
  *status = TC_OK;
  return false;
}

}  // namespace tc

extern "C" {

const char* tc_status_string(tc_status status) {
  switch (status) {
    case TC_OK: return "TC_OK";
    case TC_ERR_INVALID_ARG: return "TC_ERR_INVALID_ARG";
    case TC_ERR_ID_OUT_OF_RANGE: return "TC_ERR_ID_OUT_OF_RANGE";
    case TC_ERR_CAPACITY: return "TC_ERR_CAPACITY";
    case TC_ERR_WORKSPACE: return "TC_ERR_WORKSPACE";
    case TC_ERR_HIP: return "TC_ERR_HIP";
    case TC_ERR_UNSUPPORTED: return "TC_ERR_UNSUPPORTED";
    default: return "TC_ERR_UNKNOWN";
  }
}

const char* tc_last_error(void) { return tc::g_last_error; }

int32_t tc_version(void) { return 100; }

}  // extern "C"
