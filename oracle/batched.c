/* Oracle for the batched NLTE problem: the stationary populations of one
 * element with three ion stages per cell, under frozen rates (the linear
 * problem every fixed-point or Newton step of Sec. 2.2 solves).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The plain definition: assemble the full N x N rate matrix of the cell (all
 * stages together, as the paper solves the ion stages of one species jointly)
 * and take its stationary vector by GTH state reduction in level order, the
 * dense algorithm with no use of the matrix's structure.
 *
 * Per-level and per-pair values, Philox4x64-10 with key (seed, 6):
 *   level i of stage z in cell c: counter (c, z, i, 2^63);
 *     g = 1 + floor(9 u0), E = 0 for the ground (i = 0), else 69 kT u1, so
 *     Boltzmann factors reach e^-69 ~ 1e-30 at the cell's temperature.
 *   pair l < u of stage z in cell c: counter (c, z, l, u);
 *     radiative iff u0 < 0.2: A = 10^(-3 + 11 u1) s^-1 and
 *     Gamma_PE = gpe_table[min(n - 1, floor(u3 n))] s^-1, n = n_gpe: one of
 *     the photoexcitation rates measured from the estimators of a transport
 *     run (the stored table of the 16^3 sphere workload's rates);
 *     downward collision coefficient q = 10^(-10 + 3 u2) cm^3 s^-1.
 *   uniforms u_k = (x_k >> 11) 2^-53 of the four output words.
 * The upper level of a pair is the one with the higher energy (the higher
 * index on a tie). Rates per atom:
 *   upper -> lower: A + n_e q + (g_l/g_u) Gamma_PE       (radiative terms if radiative)
 *   lower -> upper: n_e q (g_u/g_l) exp(-(E_u - E_l)/kT) + Gamma_PE   (detailed balance)
 *   level of stage z -> ground of z+1: gamma_ion[c, z]
 *   ground of z+1 -> level i of z: n_e alpha0[z] (T/1e4)^-0.8 x
 *     (1/3 for i = 0; (2/3) g_i / sum_{j>=1} g_j otherwise).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static const double K_B = 1.380649e-16;

static double uni(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

static void draw(uint64_t seed, int64_t c, int z, uint64_t a, uint64_t b, double u[4]) {
  uint64_t ctr[4] = {(uint64_t)c, (uint64_t)z, a, b}, key[2] = {seed, 6}, out[4];
  oracle_philox4x64(ctr, key, out);
  for (int k = 0; k < 4; ++k) u[k] = uni(out[k]);
}

void oracle_batched_matrix(const or_batched* p, int64_t c, double* R) {
  const int32_t* L = p->level_count + 3 * c;
  int off[4] = {0, L[0], L[0] + L[1], L[0] + L[1] + L[2]};
  const int N = off[3];
  const double T = p->T_e[c], ne = p->n_e[c], kT = K_B * T;
  memset(R, 0, sizeof(double) * (size_t)N * N);
  double* g = malloc(sizeof(double) * N);
  double* E = malloc(sizeof(double) * N);
  for (int z = 0; z < 3; ++z)
    for (int i = 0; i < L[z]; ++i) {
      double u[4];
      draw(p->seed, c, z, (uint64_t)i, 1ull << 63, u);
      g[off[z] + i] = 1.0 + floor(9.0 * u[0]);
      E[off[z] + i] = i == 0 ? 0.0 : 69.0 * kT * u[1];
    }
  for (int z = 0; z < 3; ++z) {
    for (int l = 0; l < L[z]; ++l)
      for (int m = l + 1; m < L[z]; ++m) {
        double u[4];
        draw(p->seed, c, z, (uint64_t)l, (uint64_t)m, u);
        const int a = off[z] + l, b = off[z] + m;
        const int up = E[b] >= E[a] ? b : a, lo = up == b ? a : b;
        const int rad = u[0] < 0.2;
        const double A = rad ? pow(10.0, -3.0 + 11.0 * u[1]) : 0.0;
        int64_t it = (int64_t)(u[3] * (double)p->n_gpe);
        if (it > p->n_gpe - 1) it = p->n_gpe - 1;
        const double gam = rad ? p->gpe_table[it] : 0.0;
        const double q = pow(10.0, -10.0 + 3.0 * u[2]);
        R[up * N + lo] = A + ne * q + (g[lo] / g[up]) * gam;
        R[lo * N + up] = ne * q * (g[up] / g[lo]) * exp(-(E[up] - E[lo]) / kT) + gam;
      }
    if (z < 2 && L[z + 1] > 0) {
      const int gz1 = off[z + 1];
      double gex = 0.0;
      for (int i = 1; i < L[z]; ++i) gex += g[off[z] + i];
      const double rec = ne * p->alpha0[z] * pow(T / 1e4, -0.8);
      for (int i = 0; i < L[z]; ++i) {
        R[(off[z] + i) * N + gz1] = p->gamma_ion[2 * c + z];
        R[gz1 * N + off[z] + i] = i == 0 ? rec / 3.0 : rec * (2.0 / 3.0) * g[off[z] + i] / gex;
      }
    }
  }
  free(g);
  free(E);
}

int64_t oracle_batched(const or_batched* p, const int64_t* pop_offset, int64_t first,
                       int64_t count, int nthreads, double* pops) {
  int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : bad)
  for (int64_t c = first; c < first + count; ++c) {
    const int32_t* L = p->level_count + 3 * c;
    const int N = L[0] + L[1] + L[2];
    double* R = malloc(sizeof(double) * (size_t)N * N);
    oracle_batched_matrix(p, c, R);
    double* out = pops + pop_offset[c];
    oracle_gth(N, R, out);
    if (isnan(out[0])) ++bad;
    free(R);
  }
  return bad;
}
