// Photoionising levels, their opacity per cell and the photoionisation rates
// from the transport's tally (Sec. 2.3.1; Eq. A5). The absorption itself runs
// in the transport's event loop (transport.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "atom.hpp"
#include "common.hpp"

using namespace extrass;

struct extrass_pi_ctx {
  int device = 0;
  int N = 0, M = 0;
  std::vector<int32_t> level;   // host [M] global level, threshold order
  std::vector<double> lam;      // host [M] threshold wavelength, cm
  std::vector<double> sigma0;   // host [M] cm^2
  struct {
    int32_t* level = nullptr;   // [M]
    double* lam = nullptr;      // [M]
    double* coef = nullptr;     // [M] sigma0 / lambda^3
  } d;
};

namespace {

constexpr double kHC = 6.62607015e-27 * 2.99792458e10;  // h c, erg cm
constexpr double kSigmaKramers = 7.9e-18;                // cm^2, Eq. A5
constexpr int kMaxPiLevels = 4096;

template <class T>
hipError_t upload_vec(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// One thread per cell: a_j = n_j sigma0_j / lambda_j^3 for the plan's levels,
// and their suffix sums S_j = a_j + S_{j+1} (S_M = 0), added from the red end.
__global__ void k_pi_opacity(int64_t C, int N, int M, const int32_t* __restrict__ level,
                             const double* __restrict__ coef, const double* __restrict__ pops,
                             double* __restrict__ opac) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const double* pc = pops + c * N;
    double* row = opac + c * (2 * M + 1);
    double S = 0.0;
    row[M] = 0.0;
    for (int j = M - 1; j >= 0; --j) {
      const double n = pc[level[j]];
      const double a = n > 0.0 ? n * coef[j] : 0.0;
      row[M + 1 + j] = a;
      S = a + S;
      row[j] = S;
    }
  }
}

// One thread per cell: the prefix sums of T give each level's share of the
// full-move absorptions; Q_j adds the moves cut at the level's threshold.
__global__ void k_pi_rates(int64_t C, int N, int M, const int32_t* __restrict__ level,
                           const double* __restrict__ coef, const double* __restrict__ tally,
                           CellVolume V, double* __restrict__ gamma_pi) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const double inv_V = 1.0 / V(c);
    double* out = gamma_pi + c * N;
    for (int i = 0; i < N; ++i) out[i] = 0.0;
    const double* tc = tally + c * 2 * M;
    double pref = 0.0;
    for (int j = 0; j < M; ++j) {
      pref += tc[j];
      out[level[j]] = coef[j] * (pref + tc[M + j]) * inv_V;
    }
  }
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
}

}  // namespace

extern "C" int extrass_pi_plan_create(extrass_handle h, extrass_atom_handle a,
                                      const double* ion_energy, int32_t max_per_stage,
                                      extrass_pi_plan* out) {
  if (!h || !a || !ion_energy || !out || max_per_stage < 1)
    return fail(h, EXTRASS_EINVAL, "extrass_pi_plan_create: bad argument");
  *out = nullptr;
  struct Lv { int level; double lam, sigma0; };
  std::vector<Lv> lv;
  for (int s = 0; s < a->S; ++s) {
    const int b = a->off[s], e = a->off[s + 1];
    int top = 0;
    for (int i = b; i < e; ++i) top = std::max(top, a->lv_ion_host[i]);
    for (int z = 0; z < 2 && z < top; ++z) {
      const double E_ion = ion_energy[s * 3 + z];
      int taken = 0;
      for (int i = b; i < e && taken < max_per_stage; ++i) {
        if (a->lv_ion_host[i] != z) continue;
        const double chi = E_ion - a->lv_E_host[i];
        if (!(chi > 0.0)) continue;
        ++taken;
        lv.push_back({i, kHC / chi, kSigmaKramers / std::sqrt(chi / E_ion) / ((z + 1.0) * (z + 1.0))});
      }
    }
  }
  if (lv.empty() || (int)lv.size() > kMaxPiLevels)
    return fail(h, EXTRASS_EINVAL, "extrass_pi_plan_create: no photoionising level (or too many)");
  std::stable_sort(lv.begin(), lv.end(), [](const Lv& x, const Lv& y) { return x.lam < y.lam; });
  auto* p = new extrass_pi_ctx();
  p->device = h->device;
  p->N = a->N;
  p->M = (int)lv.size();
  std::vector<double> coef;
  for (const Lv& v : lv) {
    p->level.push_back(v.level);
    p->lam.push_back(v.lam);
    p->sigma0.push_back(v.sigma0);
    coef.push_back(v.sigma0 / (v.lam * v.lam * v.lam));
  }
  hipError_t e = hipSetDevice(h->device);
  if (e == hipSuccess) e = upload_vec(&p->d.level, p->level);
  if (e == hipSuccess) e = upload_vec(&p->d.lam, p->lam);
  if (e == hipSuccess) e = upload_vec(&p->d.coef, coef);
  if (e != hipSuccess) {
    extrass_pi_plan_destroy(p);
    return fail(h, EXTRASS_EHIP, std::string("extrass_pi_plan_create: ") + hipGetErrorString(e));
  }
  *out = p;
  return EXTRASS_OK;
}

extern "C" int extrass_pi_plan_destroy(extrass_pi_plan p) {
  if (!p) return EXTRASS_OK;
  void* ptrs[] = {p->d.level, p->d.lam, p->d.coef};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
  return EXTRASS_OK;
}

extern "C" int extrass_pi_plan_info(extrass_pi_plan p, int32_t* n_levels, int32_t* level,
                                    double* lambda_thr, double* sigma0,
                                    const double** device_lambda) {
  if (!p) return EXTRASS_EINVAL;
  if (n_levels) *n_levels = p->M;
  if (level) std::copy(p->level.begin(), p->level.end(), level);
  if (lambda_thr) std::copy(p->lam.begin(), p->lam.end(), lambda_thr);
  if (sigma0) std::copy(p->sigma0.begin(), p->sigma0.end(), sigma0);
  if (device_lambda) *device_lambda = p->d.lam;
  return EXTRASS_OK;
}

extern "C" int extrass_pi_opacity(extrass_handle h, extrass_pi_plan p, int64_t n_cells,
                                  const double* pops, double* opacity, void* stream) {
  if (!h || !p || !pops || !opacity || n_cells < 0 || p->device != h->device)
    return fail(h, EXTRASS_EINVAL, "extrass_pi_opacity: bad argument");
  if (n_cells == 0) return EXTRASS_OK;
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipLaunchKernelGGL(k_pi_opacity, dim3(grid_for(n_cells)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), n_cells, p->N, p->M, p->d.level,
                     p->d.coef, pops, opacity);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}

extern "C" int extrass_pi_rates(extrass_handle h, extrass_pi_plan p, const extrass_grid* g,
                                double t_exp, const double* tally, double* gamma_pi,
                                void* stream) {
  if (!h || !p || !g || !tally || !gamma_pi || !grid_shape_ok(g) || !(t_exp > 0.0) ||
      p->device != h->device)
    return fail(h, EXTRASS_EINVAL, "extrass_pi_rates: bad argument");
  const int64_t C = grid_cell_count(g);
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipLaunchKernelGGL(k_pi_rates, dim3(grid_for(C)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     C, p->N, p->M, p->d.level, p->d.coef, tally, grid_volumes(g, t_exp),
                     gamma_pi);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}
