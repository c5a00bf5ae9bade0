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

// Sets up the allocation-free transport's per-GPU scratch (transport.hip).
hipError_t noalloc_init(int device);

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

// Physical volume of one cell (cm^3) of an n^3 grid over [-beta_max,
// beta_max]^3 in x = v/c at time t_exp: in homologous flow position is
// v t_exp, so a cell is (2 beta_max / n) c t_exp wide.
inline double cell_volume(int n, double beta_max, double t_exp) {
  const double c_cgs = 2.99792458e10;
  const double w = 2.0 * beta_max / n * c_cgs * t_exp;
  return w * w * w;
}

template <class T>
inline size_t carve_bytes(size_t count) {
  return ((count * sizeof(T) + 255) & ~size_t(255)) + 256;
}

// ---- wave-level helpers (wave64) ----------------------------------------
// All-reductions over the 64 lanes (every lane active): within each row of 16
// lanes by DPP moves (partners lane^1, lane^2, then the mirrored lane within
// 8 and within 16), then the four row totals read from lanes 0, 16, 32, 48 and
// combined in a fixed order, so the result is the same in every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double read_lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
// A value every lane holds (a wave reduction, a per-system constant) kept in
// scalar registers: the vector registers are the scarce ones in the solvers.
__device__ __forceinline__ double uniform_d(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane 7-i within each 8
constexpr int kDppMirror = 0x140;      // lane 15-i within each 16

__device__ inline double wave_sum(double v) {
  v += dpp_mov<kDppXor1>(v);
  v += dpp_mov<kDppXor2>(v);
  v += dpp_mov<kDppHalfMirror>(v);
  v += dpp_mov<kDppMirror>(v);
  return uniform_d((read_lane_d(v, 0) + read_lane_d(v, 16)) + (read_lane_d(v, 32) + read_lane_d(v, 48)));
}
__device__ inline float wave_sum(float v) {
  v += dpp_mov<kDppXor1>(v);
  v += dpp_mov<kDppXor2>(v);
  v += dpp_mov<kDppHalfMirror>(v);
  v += dpp_mov<kDppMirror>(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}
__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_mov<kDppXor1>(v));
  v = fmax(v, dpp_mov<kDppXor2>(v));
  v = fmax(v, dpp_mov<kDppHalfMirror>(v));
  v = fmax(v, dpp_mov<kDppMirror>(v));
  return uniform_d(fmax(fmax(read_lane_d(v, 0), read_lane_d(v, 16)), fmax(read_lane_d(v, 32), read_lane_d(v, 48))));
}
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace extrass
