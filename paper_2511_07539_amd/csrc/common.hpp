// Shared host/device helpers of the extrass HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "extrass.h"

struct extrass_ctx {
  int device = 0;
  int num_cus = 256;
  std::string last_error;
  // batched NLTE launch shape per precision (0 FP64, 1 FP32): panel width and
  // work-groups per compute unit; 0 until tuned
  int batched_panel[2] = {0, 0};
  int batched_per_cu[2] = {0, 0};
};

namespace extrass {

inline int fail(extrass_handle h, int code, const std::string& what) {
  if (h) h->last_error = what;
  return code;
}

#define EXTRASS_HIP_TRY(h, call)                                                        \
  do {                                                                                  \
    hipError_t _e = (call);                                                             \
    if (_e != hipSuccess)                                                               \
      return ::extrass::fail((h), EXTRASS_EHIP,                                         \
                             std::string(#call) + ": " + hipGetErrorString(_e));        \
  } while (0)

// Carves aligned sub-buffers out of the caller's workspace.
struct Carver {
  char* base;
  size_t cap, used = 0;
  Carver(void* p, size_t c) : base(static_cast<char*>(p)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return reinterpret_cast<T*>(base + off);
  }
  bool ok() const { return used <= cap; }
};

template <class T>
inline size_t carve_bytes(size_t count) {
  return ((count * sizeof(T) + 255) & ~size_t(255)) + 256;
}

// ---- wave-level helpers (wave64) ----------------------------------------
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace extrass
