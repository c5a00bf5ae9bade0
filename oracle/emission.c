/* Oracle: deterministic emission of rays from the level populations.
 * Test infrastructure only (see oracle.h). FP64, plain loops.
 *
 * Sec. 2.3: every cell emits, for every wavelength bin (0.1 % logarithmic
 * steps) and every viewer of a grid spread evenly in polar and azimuthal
 * angle, one ray from the middle of the cell; it starts at the reddest
 * wavelength of the features in the bin (so that it cannot absorb in its own
 * line) and carries the bin's emission divided among the viewers by their
 * solid angle. The emission is the bound-bound emissivity of Eq. A3:
 * A_ul Delta E_ul beta_S N_u, beta_S from Eqs. A1-A2 at the cell's
 * populations, N_u the upper level's atoms in the cell (n_u V).
 * Readings: Delta E_ul = h c / lambda_ul (the photon energy of the line; the
 * synthetic atoms' level energies serve only detailed balance); the ray
 * weight E_bin / Delta Omega_k / E_phot, dimensionally garbled in the text, is
 * read as E_bin (Delta Omega_k / 4 pi) / E_phot, so that the rays of a bin
 * carry the bin's photons exactly once over the sphere.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define H_PLANCK 6.62607015e-27  /* erg s (exact) */
#define C_LIGHT 2.99792458e10    /* cm s^-1 (exact) */

static double beta_sobolev(double tau) { return tau <= 0.0 ? 1.0 : -expm1(-tau) / tau; }

void oracle_emission_bins(const or_atom* a, int64_t n_cells, const double* pops, double t_exp,
                          double cell_volume, const double* volumes, double lambda_min,
                          double lambda_max, int32_t n_lambda, double* bin_energy,
                          double* bin_lambda, double* outside) {
  double dlog = log(lambda_max / lambda_min);
  memset(bin_lambda, 0, sizeof(double) * (size_t)n_lambda);
  for (int32_t t = 0; t < a->n_trans; ++t) {
    double lam = a->trans_lambda[t];
    if (!(lam >= lambda_min && lam < lambda_max)) continue;
    int32_t b = (int32_t)floor(n_lambda * log(lam / lambda_min) / dlog);
    if (b < 0) b = 0;
    if (b >= n_lambda) b = n_lambda - 1;
    if (lam > bin_lambda[b]) bin_lambda[b] = lam;
  }
  for (int64_t c = 0; c < n_cells; ++c) {
    const double* n = pops + c * a->n_levels;
    const double V = volumes ? volumes[c] : cell_volume;
    double* E = bin_energy + c * n_lambda;
    memset(E, 0, sizeof(double) * (size_t)n_lambda);
    outside[c] = 0.0;
    for (int32_t t = 0; t < a->n_trans; ++t) {
      int32_t lo = a->trans_lower[t], up = a->trans_upper[t];
      double gl = a->level_g[lo], gu = a->level_g[up], lam = a->trans_lambda[t];
      double tau = a->trans_A[t] / (8.0 * M_PI) * (gu / gl) * lam * lam * lam * t_exp *
                   (n[lo] - (gl / gu) * n[up]);
      double e = a->trans_A[t] * beta_sobolev(tau) * n[up] * V * (H_PLANCK * C_LIGHT / lam);
      if (lam >= lambda_min && lam < lambda_max) {
        int32_t b = (int32_t)floor(n_lambda * log(lam / lambda_min) / dlog);
        if (b < 0) b = 0;
        if (b >= n_lambda) b = n_lambda - 1;
        E[b] += e;
      } else {
        outside[c] += e;
      }
    }
  }
}

int64_t oracle_ray_packets(int32_t n, double beta_max, const double* origins, int64_t first,
                           int64_t count, int32_t n_lambda, const double* bin_energy,
                           const double* bin_lambda, int32_t n_theta, int32_t n_phi,
                           double** packets) {
  double h = 2.0 * beta_max / n;
  int64_t cap = 1024, nr = 0;
  double* out = (double*)malloc(sizeof(double) * 8 * (size_t)cap);
  for (int64_t c = first; c < first + count; ++c) {
    double x[3];
    if (origins) {  /* the middle of the cell, given */
      for (int a = 0; a < 3; ++a) x[a] = origins[3 * (c - first) + a];
    } else {        /* the centre of the cube's cell */
      int32_t ci[3] = {(int32_t)(c % n), (int32_t)((c / n) % n), (int32_t)(c / ((int64_t)n * n))};
      for (int a = 0; a < 3; ++a) x[a] = -beta_max + (ci[a] + 0.5) * h;
    }
    for (int32_t b = 0; b < n_lambda; ++b) {
      double E = bin_energy[c * n_lambda + b];
      if (!(E > 0.0)) continue;
      double photons = E / (H_PLANCK * C_LIGHT / bin_lambda[b]);
      for (int32_t it = 0; it < n_theta; ++it) {
        double th = (it + 0.5) * M_PI / n_theta;
        double dom = (2.0 * M_PI / n_phi) * (cos(it * M_PI / n_theta) - cos((it + 1) * M_PI / n_theta));
        for (int32_t ip = 0; ip < n_phi; ++ip) {
          double ph = (ip + 0.5) * 2.0 * M_PI / n_phi;
          if (nr == cap) {
            cap *= 2;
            out = (double*)realloc(out, sizeof(double) * 8 * (size_t)cap);
          }
          double* r = out + 8 * nr++;
          r[0] = x[0];
          r[1] = x[1];
          r[2] = x[2];
          r[3] = sin(th) * cos(ph);
          r[4] = sin(th) * sin(ph);
          r[5] = cos(th);
          r[6] = bin_lambda[b];
          r[7] = photons * dom / (4.0 * M_PI);
        }
      }
    }
  }
  *packets = out;
  return nr;
}
