/* Oracle: NLTE statistical equilibrium of one species in one cell.
 * Test infrastructure only (see oracle.h). FP64, one cell at a time.
 *
 * The paper's EXCION solver (Sec. 2.2) solves all ion stages of a species
 * together as one matrix of all rates between all levels, with photoexcitation
 * rates held fixed, and iterates because the rates depend on the populations.
 * Its radiative term uses the Sobolev escape probability beta_S (Eq. A1) of
 * the line optical depth tau_S (Eq. A2), which depends on the populations.
 *
 * The plain definition computed here is the positive root n of
 *   sum_{j != i} n_j R_ji - n_i sum_{j != i} R_ij = 0  for every level i,
 *   sum_i n_i = n_species,
 * with per-atom rates R_ij (i -> j) built from (readings, see DESIGN notes in
 * the header of each helper):
 *   transition l < u (same ion stage):
 *     R_ul += A_ul beta_S(tau_ul(n)) + n_e q_ul + (g_l/g_u) Gamma_PE
 *     R_lu += n_e q_lu + Gamma_PE
 *     q_ul = 8.629e-6 Upsilon / (g_u sqrt(T)),  q_lu = q_ul (g_u/g_l) exp(-dE/kT)
 *   ionisation from every level of stage z to the ground of z+1: Gamma_ion(z);
 *   recombination from the ground of z+1 into stage z at n_e alpha_z(T),
 *     alpha_z(T) = alpha0_z (T/1e4 K)^-0.8, split 1/3 into the ground state and
 *     the rest over the excited levels by statistical weight (Appendix A.2).
 *
 * Algorithm (the root is what matters; the steps are textbook):
 *  1. cold start: Boltzmann within each stage, stage ratios from a ground-only
 *     ionisation balance;
 *  2. fixed-point steps n <- n_species * stationary(R(n)), under-relaxed in
 *     log(n), the stationary vector from the GTH algorithm (Grassmann, Taksar
 *     & Heyman 1985), which is subtraction-free and so accurate componentwise;
 *  3. Newton steps in log(n) with the analytic Jacobian, globalised by a trust
 *     radius on max |d ln n| and a decrease test on the scaled residuals. The
 *     scaled Jacobian J diag(n) is itself a generator transposed (non-negative
 *     off-diagonals, zero column sums), so the Newton system is solved by the
 *     same state-reduction elimination, pivots taken as sums of off-diagonal
 *     entries; conservation fixes the free multiple of the null vector.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#include "oracle.h"

#define K_B 1.380649e-16   /* erg/K (CODATA 2018, exact) */

/* Eq. A1 with the reading tau <= 0 -> 1 (no maser amplification). */
static double beta_s(double tau) {
  if (tau <= 0.0) return 1.0;
  return -expm1(-tau) / tau;
}

static double dbeta_s(double tau) {
  if (tau <= 0.0) return 0.0;
  if (tau < 1e-3) return -0.5 + tau * (1.0 / 3.0 - tau * (1.0 / 8.0 - tau / 30.0));
  return (exp(-tau) * (1.0 + tau) - 1.0) / (tau * tau);
}

/* Eq. A2 written as K*((g_u/g_l) n_l - n_u) with K = A lambda^3 t / (8 pi). */
static double tau_sobolev(double A, double lam, double t, double gl, double gu, double nl,
                          double nu, double* K) {
  *K = A * lam * lam * lam * t / (8.0 * M_PI);
  return *K * ((gu / gl) * nl - nu);
}

static int32_t n_stages(const or_atom* a, int32_t s) {
  int32_t z = 0;
  for (int32_t i = a->species_offset[s]; i < a->species_offset[s + 1]; ++i)
    if (a->level_ion[i] + 1 > z) z = a->level_ion[i] + 1;
  return z;
}

void oracle_rate_matrix(const or_atom* a, const or_cells* cl, int64_t c, int32_t s,
                        const double* n, double* R) {
  int32_t base = a->species_offset[s];
  int32_t Ns = a->species_offset[s + 1] - base;
  memset(R, 0, sizeof(double) * (size_t)Ns * Ns);
  double T = cl->T_e[c], ne = cl->n_e[c], kT = K_B * T;
  for (int32_t t = 0; t < a->n_trans; ++t) {
    int32_t lo = a->trans_lower[t], up = a->trans_upper[t];
    if (lo < base || lo >= base + Ns) continue;
    int32_t l = lo - base, u = up - base;
    double gl = a->level_g[lo], gu = a->level_g[up];
    double qul = 8.629e-6 * a->trans_upsilon[t] / (gu * sqrt(T));
    double qlu = qul * (gu / gl) * exp(-(a->level_energy[up] - a->level_energy[lo]) / kT);
    double K;
    double tau = tau_sobolev(a->trans_A[t], a->trans_lambda[t], cl->t_exp, gl, gu, n[l], n[u], &K);
    double gpe = cl->gamma_pe ? cl->gamma_pe[c * a->n_trans + t] : 0.0;
    R[u * Ns + l] += a->trans_A[t] * beta_s(tau) + ne * qul + (gl / gu) * gpe;
    R[l * Ns + u] += ne * qlu + gpe;
  }
  int32_t Z = n_stages(a, s);
  for (int32_t z = 0; z + 1 < Z; ++z) {
    int32_t g0 = -1, gnext = -1;
    double sumg = 0.0;
    for (int32_t i = 0; i < Ns; ++i) {
      int32_t zi = a->level_ion[base + i];
      if (zi == z && g0 < 0) g0 = i;
      else if (zi == z) sumg += a->level_g[base + i];
      if (zi == z + 1 && gnext < 0) gnext = i;
    }
    double gion = cl->gamma_ion[(c * a->n_species + s) * 3 + z];
    double rec = ne * a->ion_alpha0[s * 3 + z] * pow(T / 1e4, -0.8);
    for (int32_t i = 0; i < Ns; ++i) {
      if (a->level_ion[base + i] != z) continue;
      R[i * Ns + gnext] += gion;
      if (sumg == 0.0) {
        R[gnext * Ns + i] += rec;
      } else if (i == g0) {
        R[gnext * Ns + i] += rec / 3.0;
      } else {
        R[gnext * Ns + i] += rec * (2.0 / 3.0) * a->level_g[base + i] / sumg;
      }
    }
  }
}

/* State reduction of a generator with off-diagonal entries G (row i -> j),
 * solving x^T G = b^T (b may be NULL for the homogeneous problem), with the
 * last state's value fixed to x_last. Pivots are sums of the remaining
 * off-diagonal entries of the pivot row. G and b are overwritten. Returns 0,
 * or -1 if a pivot vanishes (reducible chain). */
static int gth_reduce_solve(int32_t N, double* G, double* b, double x_last, double* x) {
  double* S = (double*)malloc(sizeof(double) * (size_t)N);
  for (int32_t k = 0; k + 1 < N; ++k) {
    double s = 0.0;
    for (int32_t j = k + 1; j < N; ++j) s += G[k * N + j];
    if (!(s > 0.0)) { free(S); return -1; }
    S[k] = s;
    for (int32_t i = k + 1; i < N; ++i) {
      double f = G[i * N + k] / s;
      if (f == 0.0) continue;
      for (int32_t j = k + 1; j < N; ++j) {
        if (j == i) continue;
        G[i * N + j] += f * G[k * N + j];
      }
    }
    if (b) {
      for (int32_t j = k + 1; j < N; ++j) b[j] += b[k] * G[k * N + j] / s;
    }
  }
  x[N - 1] = x_last;
  for (int32_t k = N - 2; k >= 0; --k) {
    double acc = 0.0;
    for (int32_t i = k + 1; i < N; ++i) acc += x[i] * G[i * N + k];
    x[k] = (acc - (b ? b[k] : 0.0)) / S[k];
  }
  free(S);
  return 0;
}

void oracle_gth(int32_t N, const double* R, double* pi) {
  double* G = (double*)malloc(sizeof(double) * (size_t)N * N);
  memcpy(G, R, sizeof(double) * (size_t)N * N);
  for (int32_t i = 0; i < N; ++i) G[i * N + i] = 0.0;
  if (gth_reduce_solve(N, G, NULL, 1.0, pi) != 0) {
    for (int32_t i = 0; i < N; ++i) pi[i] = NAN;
  } else {
    double s = 0.0;
    for (int32_t i = 0; i < N; ++i) s += pi[i];
    for (int32_t i = 0; i < N; ++i) pi[i] /= s;
  }
  free(G);
}

void oracle_nlte_cold(const or_atom* a, const or_cells* cl, int64_t c, double* out) {
  double T = cl->T_e[c], ne = cl->n_e[c], kT = K_B * T;
  for (int32_t s = 0; s < a->n_species; ++s) {
    int32_t base = a->species_offset[s];
    int32_t Ns = a->species_offset[s + 1] - base;
    int32_t Z = n_stages(a, s);
    double ratio[3] = {1.0, 1.0, 1.0}, stage_sum[3] = {0, 0, 0};
    for (int32_t z = 1; z < Z; ++z) {
      double gion = cl->gamma_ion[(c * a->n_species + s) * 3 + (z - 1)];
      double rec = ne * a->ion_alpha0[s * 3 + (z - 1)] * pow(T / 1e4, -0.8);
      double r = rec > 0.0 ? gion / rec : 1e30;
      if (r < 1e-30) r = 1e-30;
      if (r > 1e30) r = 1e30;
      ratio[z] = ratio[z - 1] * r;
    }
    for (int32_t i = 0; i < Ns; ++i) {
      double w = a->level_g[base + i] * exp(-a->level_energy[base + i] / kT);
      if (w < 1e-250) w = 1e-250;
      out[base + i] = w;
      stage_sum[a->level_ion[base + i]] += w;
    }
    double rsum = 0.0;
    for (int32_t z = 0; z < Z; ++z) rsum += ratio[z];
    double ntot = cl->n_species[c * a->n_species + s];
    for (int32_t i = 0; i < Ns; ++i) {
      int32_t z = a->level_ion[base + i];
      out[base + i] = ntot * (ratio[z] / rsum) * (out[base + i] / stage_sum[z]);
    }
  }
}

/* One species of one cell. n (local numbering, length Ns) holds the start on
 * entry and the solution on exit. Returns the iteration count, or -1.
 *
 * Step 1: fixed-point steps n <- n_species * stationary(R(n)), under-relaxed
 *   in log(n), until the change is below 0.1 in log (at most 60 steps).
 * Step 2: Newton on the level equations in log(n): the correction
 *   delta = d ln n solves J diag(n) delta = -F with sum n_i delta_i fixed by
 *   conservation, and the update is n_i exp(delta_i) (positive by
 *   construction). -F is formed as Q(n)^T (P(n) - n), P(n) being the
 *   GTH stationary vector of the current rates scaled to n_species: the
 *   same vector, free of the cancellation between gross inflow and outflow
 *   that limits a directly summed F to ~1e-9 in weakly coupled stages. Far
 *   from the root the step is limited to a trust radius (max |delta_i| <=
 *   Delta) and accepted only if it lowers sum_i (P(n)_i/n_i - 1)^2; a
 *   rejected step shrinks the radius.
 * Converged when max |delta| < tol and max |P(n)_i/n_i - 1| < 1e-10, or when
 * max |delta| < 1e-11 has not improved for 3 steps, or when no step lowers the
 * fixed-point residual any more and it is at rounding level.
 */
static int solve_species(const or_atom* a, const or_cells* cl, int64_t c, int32_t s, double* n,
                         int max_iter, double tol) {
  int32_t base = a->species_offset[s];
  int32_t Ns = a->species_offset[s + 1] - base;
  double ntot = cl->n_species[c * a->n_species + s];
  size_t NN = (size_t)Ns * Ns;
  double* R = (double*)malloc(sizeof(double) * NN);
  double* G = (double*)malloc(sizeof(double) * NN);
  double* Gp = (double*)malloc(sizeof(double) * NN);
  double* b = (double*)malloc(sizeof(double) * Ns);
  double* bp = (double*)malloc(sizeof(double) * Ns);
  double* x = (double*)malloc(sizeof(double) * Ns);
  double* pi = (double*)malloc(sizeof(double) * Ns);
  double* trial = (double*)malloc(sizeof(double) * Ns);
  double* wscale = (double*)malloc(sizeof(double) * Ns);
  double* hres = (double*)malloc(sizeof(double) * Ns);
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * Ns);
  int it, result = -1, best_it = 0;
  double Delta = 1.0, best_step = INFINITY;

  /* fixed-point phase, under-relaxed in log(n): omega halves whenever the
   * change fails to shrink (this also breaks period-2 cycles) and never grows
   * back; ends once max |d ln n| < 0.1 */
  {
    double omega = 1.0, prev = INFINITY;
    for (it = 0; it < max_iter && it < 60; ++it) {
      oracle_rate_matrix(a, cl, c, s, n, R);
      oracle_gth(Ns, R, pi);
      if (!(pi[0] == pi[0])) goto out;
      double change = 0.0;
      for (int32_t i = 0; i < Ns; ++i) {
        double d = fabs(log(ntot * pi[i] / n[i]));
        if (d > change) change = d;
      }
      if (change > 0.999 * prev) omega = omega * 0.5 > 1.0 / 1024 ? omega * 0.5 : 1.0 / 1024;
      prev = change;
      double tot = 0.0;
      for (int32_t i = 0; i < Ns; ++i) {
        n[i] = exp((1.0 - omega) * log(n[i]) + omega * log(ntot * pi[i]));
        tot += n[i];
      }
      for (int32_t i = 0; i < Ns; ++i) n[i] *= ntot / tot;
      if (change < 0.1) { ++it; break; }
    }
  }

  int have_p = 0;
  for (; it < max_iter; ++it) {
    /* Fixed-point residual h_i = P(n)_i / n_i - 1, with P(n) = n_species *
     * stationary(R(n)) from GTH: no cancellation, accurate componentwise. */
    if (!have_p) {
      oracle_rate_matrix(a, cl, c, s, n, R);
      oracle_gth(Ns, R, pi);
      if (!(pi[0] == pi[0])) goto out;
      for (int32_t i = 0; i < Ns; ++i) hres[i] = ntot * pi[i] / n[i] - 1.0;
    }
    double res = 0.0, phi = 0.0;
    for (int32_t i = 0; i < Ns; ++i) {
      if (fabs(hres[i]) > res) res = fabs(hres[i]);
      phi += hres[i] * hres[i];
    }
    /* Newton right-hand side -F(n) written as Q(n)^T (P(n) - n): with the flux
     * matrix G_ij = n_i R_ij, (Q^T H)_i = sum_j h_j G_ji - h_i sum_j G_ij. It is
     * the same vector as -F, formed from the small h instead of the cancelling
     * gross inflows and outflows. */
    oracle_rate_matrix(a, cl, c, s, n, R);
    for (size_t e = 0; e < NN; ++e) G[e] = 0.0;
    for (int32_t k = 0; k < Ns; ++k)
      for (int32_t j = 0; j < Ns; ++j)
        if (j != k) G[k * Ns + j] = n[k] * R[k * Ns + j];
    for (int32_t i = 0; i < Ns; ++i) {
      double in = 0.0, outr = 0.0;
      for (int32_t j = 0; j < Ns; ++j) {
        if (j == i) continue;
        in += hres[j] * G[j * Ns + i];
        outr += G[i * Ns + j];
      }
      b[i] = in - hres[i] * outr;
    }
    /* scaled Jacobian as a generator: G_kj = n_k dF_j/dn_k (k != j) */
    for (int32_t t = 0; t < a->n_trans; ++t) {
      int32_t lo = a->trans_lower[t], up = a->trans_upper[t];
      if (lo < base || lo >= base + Ns) continue;
      int32_t l = lo - base, u = up - base;
      double gl = a->level_g[lo], gu = a->level_g[up], K;
      double tau = tau_sobolev(a->trans_A[t], a->trans_lambda[t], cl->t_exp, gl, gu, n[l], n[u], &K);
      double db = dbeta_s(tau);
      if (db == 0.0) continue;
      double du = -n[u] * a->trans_A[t] * db * K;            /* d flux / d n_u, >= 0 */
      double dl = n[u] * a->trans_A[t] * db * K * (gu / gl);  /* d flux / d n_l, <= 0 */
      G[u * Ns + l] += du * n[u];
      G[l * Ns + u] += -dl * n[l];
    }
    /* The state eliminated last (its value fixed, then set by conservation)
     * is the most populated level, so that the normalisation is carried by the
     * level that dominates the sum. */
    {
      int32_t big = 0;
      for (int32_t i = 1; i < Ns; ++i) if (n[i] > n[big]) big = i;
      for (int32_t i = 0; i < Ns; ++i) perm[i] = i;
      perm[big] = Ns - 1;
      perm[Ns - 1] = big;
      for (int32_t i = 0; i < Ns; ++i) {
        bp[i] = b[perm[i]];
        for (int32_t j = 0; j < Ns; ++j) Gp[i * Ns + j] = G[perm[i] * Ns + perm[j]];
      }
    }
    if (gth_reduce_solve(Ns, Gp, bp, 0.0, x) != 0) goto out;
    /* homogeneous solution of the same reduced system */
    pi[Ns - 1] = 1.0;
    for (int32_t k = Ns - 2; k >= 0; --k) {
      double acc = 0.0, sk = 0.0;
      for (int32_t j = k + 1; j < Ns; ++j) sk += Gp[k * Ns + j];
      for (int32_t i = k + 1; i < Ns; ++i) acc += pi[i] * Gp[i * Ns + k];
      pi[k] = acc / sk;
    }
    /* back to level order */
    for (int32_t i = 0; i < Ns; ++i) { bp[perm[i]] = x[i]; trial[perm[i]] = pi[i]; }
    double sum_n = 0.0, sum_nx = 0.0, sum_npi = 0.0;
    for (int32_t i = 0; i < Ns; ++i) {
      x[i] = bp[i];
      pi[i] = trial[i];
      sum_n += n[i];
      sum_nx += n[i] * x[i];
      sum_npi += n[i] * pi[i];
    }
    double cst = ((ntot - sum_n) - sum_nx) / sum_npi;
    double step = 0.0;
    for (int32_t i = 0; i < Ns; ++i) {
      x[i] += cst * pi[i];
      if (fabs(x[i]) > step) step = fabs(x[i]);
    }
    if (step < best_step) { best_step = step; best_it = it; }
    if ((step < tol && res < 1e-10) || (step < 1e-11 && it - best_it >= 3)) {
      result = it + 1;
      goto out;
    }
    /* trust-region step in log(n), accepted when the fixed-point residual drops */
    int accepted = 0;
    double taken = 0.0;
    for (int bt = 0; bt < 40; ++bt) {
      double scale = step > Delta ? Delta / step : 1.0;
      double tot = 0.0;
      taken = step * scale;
      for (int32_t i = 0; i < Ns; ++i) {
        trial[i] = n[i] * exp(scale * x[i]);
        tot += trial[i];
      }
      for (int32_t i = 0; i < Ns; ++i) trial[i] *= ntot / tot;
      oracle_rate_matrix(a, cl, c, s, trial, R);
      oracle_gth(Ns, R, pi);
      double phi2 = 0.0, res2 = 0.0;
      for (int32_t i = 0; i < Ns; ++i) {
        double hv = ntot * pi[i] / trial[i] - 1.0;
        wscale[i] = hv;
        phi2 += hv * hv;
        if (fabs(hv) > res2) res2 = fabs(hv);
      }
      if (phi2 < phi || res2 < 1e-14) { accepted = 1; break; }
      Delta = (taken < Delta ? taken : Delta) / 4.0;
    }
    if (!accepted) {
      if (step < 1e-11 || res < 1e-14) result = it + 1; /* stalled at rounding level */
      goto out;
    }
    for (int32_t i = 0; i < Ns; ++i) { n[i] = trial[i]; hres[i] = wscale[i]; }
    have_p = 1;
    if (taken >= 0.99 * Delta) Delta = 2.0 * Delta < 30.0 ? 2.0 * Delta : 30.0;
  }
out:
  free(R); free(G); free(Gp); free(b); free(bp); free(x); free(pi); free(trial); free(perm); free(wscale); free(hres);
  return result;
}

int oracle_nlte(const or_atom* a, const or_cells* cl, int64_t first, int64_t count, int use_guess,
                int max_iter, double tol, int nthreads, double* pops, int32_t* status,
                int32_t* iters) {
  if (nthreads < 1) nthreads = 1;
  int32_t N = a->n_levels;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
  for (int64_t c = first; c < first + count; ++c) {
    double* pc = pops + c * N;
    int empty = 1;
    for (int32_t s = 0; s < a->n_species; ++s)
      if (cl->n_species[c * a->n_species + s] > 0.0) empty = 0;
    if (empty) {
      for (int32_t i = 0; i < N; ++i) pc[i] = 0.0;
      status[c] = 3;
      if (iters) iters[c] = 0;
      continue;
    }
    if (!use_guess) oracle_nlte_cold(a, cl, c, pc);
    int st = 0, itmax = 0;
    for (int32_t s = 0; s < a->n_species; ++s) {
      if (!(cl->n_species[c * a->n_species + s] > 0.0)) continue;
      int r = solve_species(a, cl, c, s, pc + a->species_offset[s], max_iter, tol);
      if (r < 0) st = 2;
      else if (r > itmax) itmax = r;
    }
    status[c] = st;
    if (iters) iters[c] = itmax;
  }
  return 0;
}
