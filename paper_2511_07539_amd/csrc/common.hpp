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

// The cells' volumes of a grid: one value for the cube, or per cell from the
// edges of a spherical grid, (r_b^3 - r_a^3)/3 (cos theta_a - cos theta_b)
// (2 pi / n_phi) (c t)^3 for cell c = i_r + n_r (i_theta + n_theta i_phi).
struct CellVolume {
  double cube = 0.0;            // the cube's cell volume (sph == false)
  bool sph = false;
  int nr = 0, nt = 0, np = 0;
  const double* r = nullptr;    // device [nr + 1]
  const double* th = nullptr;   // device [nt + 1]
  double ct3 = 0.0;             // (c t)^3
  __device__ double operator()(int64_t c) const {
    if (!sph) return cube;
    const int ir = (int)(c % nr);
    const int it = (int)((c / nr) % nt);
    const double ra = r[ir], rb = r[ir + 1];
    return (rb * rb * rb - ra * ra * ra) / 3.0 * (cos(th[it]) - cos(th[it + 1])) *
           (2.0 * M_PI / np) * ct3;
  }
};

// The grid's cell count and volumes at time t_exp (host).
inline int64_t grid_cell_count(const extrass_grid* g) {
  if (g->spherical)
    return (int64_t)g->spherical->n_r * g->spherical->n_theta * g->spherical->n_phi;
  return (int64_t)g->n * g->n * g->n;
}

inline CellVolume grid_volumes(const extrass_grid* g, double t_exp) {
  CellVolume v;
  if (g->spherical) {
    const double ct = 2.99792458e10 * t_exp;
    v.sph = true;
    v.nr = g->spherical->n_r;
    v.nt = g->spherical->n_theta;
    v.np = g->spherical->n_phi;
    v.r = g->spherical->r_edge;
    v.th = g->spherical->theta_edge;
    v.ct3 = ct * ct * ct;
  } else {
    v.cube = cell_volume(g->n, g->beta_max, t_exp);
  }
  return v;
}

// A grid's shape is valid: a cube of 1..1024 cells per axis with beta_max > 0,
// or a spherical grid with every count >= 1, edge arrays and C < 2^31.
inline bool grid_shape_ok(const extrass_grid* g) {
  if (g->spherical) {
    const extrass_spherical* p = g->spherical;
    return p->n_r >= 1 && p->n_theta >= 1 && p->n_phi >= 1 && p->r_edge && p->theta_edge &&
           (int64_t)p->n_r * p->n_theta * p->n_phi <= 2147483647LL;
  }
  return g->n > 0 && g->n <= 1024 && g->beta_max > 0.0;
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
