// Line emission of every cell for the deterministic rays (Sec. 2.3; Eq. A3):
// the bound-bound emissivity A_ul (h c / lambda_ul) beta_S N_u of each atom
// transition, binned by wavelength into the bins a plan fixes for the atom.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "atom.hpp"
#include "common.hpp"

using namespace extrass;

struct extrass_emission_ctx {
  int device = 0;
  int T = 0, B = 0;
  double lambda_min = 0, lambda_max = 0;
  int n_lambda = 0;
  std::vector<int32_t> bin_number;  // host [B]
  std::vector<double> bin_lambda;   // host [B]
  struct {
    int32_t* slot_start = nullptr;  // [B+1] transitions of slot j: slot_trans[start[j] .. start[j+1])
    int32_t* slot_trans = nullptr;  // [T_in]
    int32_t* out_trans = nullptr;   // [T_out] transitions outside the range
    double* bin_lambda = nullptr;   // [B]
  } d;
  int T_out = 0;
};

namespace {

constexpr double kHC = 6.62607015e-27 * 2.99792458e10;  // h c, erg cm

template <class T>
hipError_t upload_vec(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// A_ul beta_S(tau_ul) n_u of transition t at the cell's populations (Eqs. A1,
// A2): decays per second per unit volume that escape the line.
__device__ __forceinline__ double escaping_decays(const extrass_atom_ctx::Dev& d, int t,
                                                  const double* pc, double t_exp) {
  const double nl = pc[d.o_lo[t]], nu = pc[d.o_up[t]];
  const double tau = d.o_K[t] * t_exp * (nl - d.o_r[t] * nu);
  const double beta = tau <= 0.0 ? 1.0 : -expm1(-tau) / tau;
  return d.o_A[t] * beta * nu;
}

// One thread per (cell, occupied bin): photons s^-1 the cell emits in the
// bin, sum over its transitions of A beta n_u V (lambda_bin / lambda_t) (the
// bin's energy over the photon energy h c / lambda_bin). One thread per cell
// for the energy of the lines outside the range.
__global__ void k_emission(int64_t C, int N, int B, extrass_atom_ctx::Dev d,
                           const int32_t* __restrict__ slot_start,
                           const int32_t* __restrict__ slot_trans,
                           const double* __restrict__ bin_lambda, const double* __restrict__ pops,
                           double t_exp, CellVolume V, double* __restrict__ bin_photons) {
  const int64_t total = C * B;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / B;
    const int j = static_cast<int>(e - c * B);
    const double* pc = pops + c * N;
    double acc = 0.0;
    for (int i = slot_start[j]; i < slot_start[j + 1]; ++i) {
      const int t = slot_trans[i];
      acc += escaping_decays(d, t, pc, t_exp) * (bin_lambda[j] / d.o_lam[t]);
    }
    bin_photons[e] = acc * V(c);
  }
}

__global__ void k_emission_outside(int64_t C, int N, int n_out, extrass_atom_ctx::Dev d,
                                   const int32_t* __restrict__ out_trans,
                                   const double* __restrict__ pops, double t_exp, CellVolume V,
                                   double* __restrict__ outside) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const double* pc = pops + c * N;
    double acc = 0.0;
    for (int i = 0; i < n_out; ++i) {
      const int t = out_trans[i];
      acc += escaping_decays(d, t, pc, t_exp) * (kHC / d.o_lam[t]);
    }
    outside[c] = acc * V(c);
  }
}

}  // namespace

extern "C" int extrass_emission_plan_create(extrass_handle h, extrass_atom_handle a,
                                            double lambda_min, double lambda_max,
                                            int32_t n_lambda, extrass_emission_plan* out) {
  if (!h || !a || !out || !(lambda_min > 0.0) || !(lambda_max > lambda_min) || n_lambda < 1 ||
      n_lambda > (1 << 24))
    return fail(h, EXTRASS_EINVAL, "extrass_emission_plan_create: bad argument");
  *out = nullptr;
  auto* p = new extrass_emission_ctx();
  p->device = h->device;
  p->T = a->T;
  p->lambda_min = lambda_min;
  p->lambda_max = lambda_max;
  p->n_lambda = n_lambda;
  const double dlog = std::log(lambda_max / lambda_min);
  // bin of each transition inside the range; the occupied bins in order
  std::vector<int> bin(a->T, -1);
  std::vector<int32_t> out_t;
  for (int t = 0; t < a->T; ++t) {
    const double lam = a->lam_host[t];
    if (lam >= lambda_min && lam < lambda_max) {
      int b = static_cast<int>(std::floor(n_lambda * std::log(lam / lambda_min) / dlog));
      bin[t] = std::min(std::max(b, 0), n_lambda - 1);
    } else {
      out_t.push_back(t);
    }
  }
  std::vector<int32_t> order;
  for (int t = 0; t < a->T; ++t)
    if (bin[t] >= 0) order.push_back(t);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return bin[x] < bin[y]; });
  std::vector<int32_t> start{0};
  for (size_t i = 0; i < order.size(); ++i) {
    const int t = order[i];
    if (i == 0 || bin[t] != bin[order[i - 1]]) {
      if (i > 0) start.push_back(static_cast<int32_t>(i));
      p->bin_number.push_back(bin[t]);
      p->bin_lambda.push_back(a->lam_host[t]);
    }
    p->bin_lambda.back() = std::max(p->bin_lambda.back(), a->lam_host[t]);
  }
  start.push_back(static_cast<int32_t>(order.size()));
  if (order.empty()) start.assign(1, 0);
  p->B = static_cast<int>(p->bin_number.size());
  p->T_out = static_cast<int>(out_t.size());
  hipError_t e = hipSetDevice(h->device);
  if (e == hipSuccess) e = upload_vec(&p->d.slot_start, start);
  if (e == hipSuccess) e = upload_vec(&p->d.slot_trans, order);
  if (e == hipSuccess) e = upload_vec(&p->d.out_trans, out_t);
  if (e == hipSuccess) e = upload_vec(&p->d.bin_lambda, p->bin_lambda);
  if (e != hipSuccess) {
    extrass_emission_plan_destroy(p);
    return fail(h, EXTRASS_EHIP, std::string("extrass_emission_plan_create: ") + hipGetErrorString(e));
  }
  *out = p;
  return EXTRASS_OK;
}

extern "C" int extrass_emission_plan_destroy(extrass_emission_plan p) {
  if (!p) return EXTRASS_OK;
  void* ptrs[] = {p->d.slot_start, p->d.slot_trans, p->d.out_trans, p->d.bin_lambda};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
  return EXTRASS_OK;
}

extern "C" int extrass_emission_plan_info(extrass_emission_plan p, int32_t* n_bins,
                                          int32_t* bin_number, double* bin_lambda,
                                          const double** device_lambda) {
  if (!p) return EXTRASS_EINVAL;
  if (n_bins) *n_bins = p->B;
  if (bin_number) std::copy(p->bin_number.begin(), p->bin_number.end(), bin_number);
  if (bin_lambda) std::copy(p->bin_lambda.begin(), p->bin_lambda.end(), bin_lambda);
  if (device_lambda) *device_lambda = p->d.bin_lambda;
  return EXTRASS_OK;
}

extern "C" int extrass_emission(extrass_handle h, extrass_emission_plan p, extrass_atom_handle a,
                                const extrass_grid* g, double t_exp, const double* pops,
                                double* bin_photons, double* outside, void* stream) {
  if (!h || !p || !a || !g || !pops || !bin_photons || !grid_shape_ok(g) || !(t_exp > 0.0) ||
      p->T != a->T || p->device != h->device)
    return fail(h, EXTRASS_EINVAL, "extrass_emission: bad argument");
  const int64_t C = grid_cell_count(g);
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const CellVolume V = grid_volumes(g, t_exp);
  if (p->B > 0) {
    const int64_t blocks = std::min<int64_t>((C * p->B + 255) / 256, 65536);
    hipLaunchKernelGGL(k_emission, dim3((unsigned)blocks), dim3(256), 0, st, C, a->N, p->B, a->d,
                       p->d.slot_start, p->d.slot_trans, p->d.bin_lambda, pops, t_exp, V,
                       bin_photons);
  }
  if (outside) {
    const int64_t blocks = std::min<int64_t>((C + 255) / 256, 65536);
    hipLaunchKernelGGL(k_emission_outside, dim3((unsigned)blocks), dim3(256), 0, st, C, a->N,
                       p->T_out, a->d, p->d.out_trans, pops, t_exp, V, outside);
  }
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}
