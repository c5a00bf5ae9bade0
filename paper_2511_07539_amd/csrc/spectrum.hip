// Emergent spectra per viewer (Sec. 2.3: rays leave towards 20 x 20 viewers
// spread evenly in polar and azimuthal angle, the emergent emission is binned
// logarithmically in wavelength, and global convergence compares the energy
// in the emergent spectra with the deposition).
//
// One thread per packet record: an escaped packet's weight (and energy
// w h c / lambda_L) goes to the bin of its viewer (theta, phi of its lab-frame
// direction, which a ray keeps in homologous flow) and of its lab wavelength.
// Escaped packets are a few per cent of the packets, so the atomics are few;
// the launch is bound by reading the 64-byte records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "extrass.h"

namespace extrass {
namespace {

constexpr double kPlanck = 6.62607015e-27;  // erg s
constexpr double kLight = 2.99792458e10;    // cm s^-1

struct SpecArgs {
  const double* pk;
  int64_t P;
  int n_theta, n_phi, n_lambda;
  double lam_min, lam_max;
  double* photons;
  double* energy;
};

__global__ void k_spectrum(SpecArgs A) {
  const double two_pi = 2.0 * M_PI;
  const double inv_dlog = (double)A.n_lambda / log(A.lam_max / A.lam_min);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A.P;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double* r = A.pk + (int64_t)EXTRASS_PACKET_FIELDS * i;
    const double w = r[0];
    if (!(w > 0.0)) continue;  // stopped in the grid (or never written)
    const double lam = r[1];
    if (!(lam >= A.lam_min && lam < A.lam_max)) continue;
    int b = (int)floor(log(lam / A.lam_min) * inv_dlog);
    b = b < 0 ? 0 : (b >= A.n_lambda ? A.n_lambda - 1 : b);
    const double nz = fmin(1.0, fmax(-1.0, r[6]));
    int it = (int)floor(acos(nz) * (A.n_theta / M_PI));
    it = it < 0 ? 0 : (it >= A.n_theta ? A.n_theta - 1 : it);
    double phi = atan2(r[5], r[4]);
    if (phi < 0.0) phi += two_pi;
    int ip = (int)floor(phi * (A.n_phi / two_pi));
    ip = ip < 0 ? 0 : (ip >= A.n_phi ? A.n_phi - 1 : ip);
    const int64_t at = ((int64_t)it * A.n_phi + ip) * A.n_lambda + b;
    if (A.photons) atomicAdd(A.photons + at, w);
    if (A.energy) atomicAdd(A.energy + at, w * (kPlanck * kLight / lam));
  }
}

}  // namespace
}  // namespace extrass

using namespace extrass;

extern "C" int extrass_spectrum(extrass_handle h, const double* packets, int64_t n_packets,
                                const extrass_spectrum_bins* bins, double* photons,
                                double* energy, void* stream) {
  if (!h || !bins || n_packets < 0 || (n_packets > 0 && !packets))
    return fail(h, EXTRASS_EINVAL, "extrass_spectrum: bad argument");
  const extrass_spectrum_bins& sb = *bins;
  if (sb.n_theta < 1 || sb.n_theta > 4096 || sb.n_phi < 1 || sb.n_phi > 4096 || sb.n_lambda < 1 ||
      sb.n_lambda > (1 << 20) || !(sb.lambda_min > 0.0) || !(sb.lambda_max > sb.lambda_min) ||
      !std::isfinite(sb.lambda_max))
    return fail(h, EXTRASS_EINVAL, "extrass_spectrum: bad bins");
  if (n_packets == 0 || (!photons && !energy)) return EXTRASS_OK;
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  SpecArgs A{packets, n_packets, sb.n_theta, sb.n_phi, sb.n_lambda, sb.lambda_min, sb.lambda_max,
             photons, energy};
  const int64_t blocks = std::min<int64_t>((n_packets + 255) / 256, (int64_t)h->num_cus * 16);
  hipLaunchKernelGGL(k_spectrum, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), A);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}
