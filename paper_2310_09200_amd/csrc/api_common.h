// Host-side pieces shared by the translation units of the C ABI: the context
// object, workspace alignment, error reporting and the HIP status check.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "bluebild.h"

struct bb_context_ {
  int device = 0;
  hipStream_t stream = nullptr;
  rocblas_handle rb = nullptr;
  std::string err;
  int live = 0;
  // device address of the library's fixed scratch on this device (looked up
  // when the context is created; used by bb_synth_collect_eig_noalloc)
  void* noalloc_scratch = nullptr;
  // device architecture name without feature suffixes ("gfx950"): the key of
  // the autotune cache entries
  std::string arch;
};

namespace bb_host {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline bb_status fail(bb_context ctx, bb_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return s;
}

inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Debug aid: with BB_DEBUG_FILL set (and not "0") in the environment, the
// library fills every workspace it is given with 0xFF bytes (a NaN in float32
// and float64, -1 in integers) before using it, so that a read of workspace
// memory that no kernel wrote shows up in the results.
inline bool debug_fill() {
  const char* v = std::getenv("BB_DEBUG_FILL");
  return v && v[0] && !(v[0] == '0' && v[1] == 0);
}

}  // namespace bb_host

#define BB_HIP(ctx, call)                                                                                      \
  do {                                                                                                         \
    hipError_t e_ = (call);                                                                                    \
    if (e_ != hipSuccess) return bb_host::fail((ctx), BB_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)
