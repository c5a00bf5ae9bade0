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
 * with per-atom rates R_ij (i -> j) built from (where the paper is silent,
 * the reading taken is stated beside the formula):
 *   transition l < u (same ion stage):
 *     R_ul += A_ul beta_S(tau_ul(n)) + n_e q_ul + (g_l/g_u) Gamma_PE
 *     R_lu += n_e q_lu + Gamma_PE
 *     q_ul = 8.629e-6 Upsilon / (g_u sqrt(T)),  q_lu = q_ul (g_u/g_l) exp(-dE/kT)
 *   ionisation from every level of stage z to the ground of z+1: Gamma_ion(z);
 *   recombination from the ground of z+1 into stage z at n_e alpha_z(T),
 *     alpha_z(T) = alpha0_z (T/1e4 K)^-0.8, split 1/3 into the ground state and
 *     the rest over the excited levels by statistical weight (Appendix A.2).
 *
 * Algorithm (solve_species below): the paper's damped Newton-Raphson with a
 * numerical Jacobian brings the populations close to the root; a fixed-point
 * iteration on the stationary vector of the rates (GTH, componentwise
 * accurate) finishes the solve, and only a root test ends it.
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

/* Every rate of species s in cell c that does not depend on the populations
 * (R[i*Ns+j], i -> j, per atom in i): collisions, photoexcitation and
 * photo-de-excitation, ionisation (the stage's rate plus each level's
 * photoionisation rate, when given) and recombination. The radiative decay
 * A beta_S(tau(n)) is added by add_decay. */
static void rates_without_decay(const or_atom* a, const or_cells* cl, int64_t c, int32_t s,
                                double* R) {
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
    double gpe = cl->gamma_pe ? cl->gamma_pe[c * a->n_trans + t] : 0.0;
    R[u * Ns + l] += ne * qul + (gl / gu) * gpe;
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
      /* stage ionisation rate plus the level's own photoionisation (Sec. 2.3.1) */
      R[i * Ns + gnext] += gion + (cl->gamma_pi ? cl->gamma_pi[c * a->n_levels + base + i] : 0.0);
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

/* Adds the radiative decay A_ul beta_S(tau_ul(n)) of every transition of
 * species s (Eqs. A1, A2) to R at the populations n (species-local). */
static void add_decay(const or_atom* a, const or_cells* cl, int32_t s, const double* n,
                      double* R) {
  int32_t base = a->species_offset[s];
  int32_t Ns = a->species_offset[s + 1] - base;
  for (int32_t t = 0; t < a->n_trans; ++t) {
    int32_t lo = a->trans_lower[t], up = a->trans_upper[t];
    if (lo < base || lo >= base + Ns) continue;
    int32_t l = lo - base, u = up - base;
    double K;
    double tau = tau_sobolev(a->trans_A[t], a->trans_lambda[t], cl->t_exp, a->level_g[lo],
                             a->level_g[up], n[l], n[u], &K);
    R[u * Ns + l] += a->trans_A[t] * beta_s(tau);
  }
}

void oracle_rate_matrix(const or_atom* a, const or_cells* cl, int64_t c, int32_t s,
                        const double* n, double* R) {
  rates_without_decay(a, cl, c, s, R);
  add_decay(a, cl, s, n, R);
}

/* Stationary vector of a continuous-time Markov chain by state reduction
 * (Grassmann, Taksar & Heyman 1985): R holds the off-diagonal rates (row
 * i -> j; the diagonal is ignored). States are eliminated in index order,
 * each pivot being the sum of the remaining off-diagonal rates of its row,
 * so no subtraction occurs. pi sums to 1; NaN if a pivot vanishes
 * (reducible chain). */
void oracle_gth(int32_t N, const double* R, double* pi) {
  double* G = (double*)malloc(sizeof(double) * (size_t)N * N);
  double* S = (double*)malloc(sizeof(double) * (size_t)N);
  memcpy(G, R, sizeof(double) * (size_t)N * N);
  for (int32_t i = 0; i < N; ++i) G[i * N + i] = 0.0;
  int ok = 1;
  for (int32_t k = 0; k + 1 < N && ok; ++k) {
    double s = 0.0;
    for (int32_t j = k + 1; j < N; ++j) s += G[k * N + j];
    if (!(s > 0.0)) { ok = 0; break; }
    S[k] = s;
    /* The update also reaches the diagonal G[i][i], which no later step
     * reads: pivots sum only the entries right of the diagonal, and the
     * back-substitution only those left of it. */
    for (int32_t i = k + 1; i < N; ++i) {
      double f = G[i * N + k] / s;
      if (f == 0.0) continue;
      for (int32_t j = k + 1; j < N; ++j) G[i * N + j] += f * G[k * N + j];
    }
  }
  if (ok) {
    pi[N - 1] = 1.0;
    for (int32_t k = N - 2; k >= 0; --k) {
      double acc = 0.0;
      for (int32_t i = k + 1; i < N; ++i) acc += pi[i] * G[i * N + k];
      pi[k] = acc / S[k];
    }
    double s = 0.0;
    for (int32_t i = 0; i < N; ++i) s += pi[i];
    for (int32_t i = 0; i < N; ++i) pi[i] /= s;
  } else {
    for (int32_t i = 0; i < N; ++i) pi[i] = NAN;
  }
  free(G);
  free(S);
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

/* Solves M x = b (M is N x N, row-major) by Gaussian elimination with
 * partial pivoting; M and b are overwritten. Returns -1 if M is singular. */
static int gauss_solve(int32_t N, double* M, double* b, double* x) {
  for (int32_t k = 0; k < N; ++k) {
    int32_t p = k;
    for (int32_t i = k + 1; i < N; ++i)
      if (fabs(M[i * N + k]) > fabs(M[p * N + k])) p = i;
    if (!(M[p * N + k] != 0.0)) return -1;
    if (p != k) {
      for (int32_t j = 0; j < N; ++j) {
        double t = M[k * N + j]; M[k * N + j] = M[p * N + j]; M[p * N + j] = t;
      }
      double t = b[k]; b[k] = b[p]; b[p] = t;
    }
    for (int32_t i = k + 1; i < N; ++i) {
      double f = M[i * N + k] / M[k * N + k];
      if (f == 0.0) continue;
      for (int32_t j = k; j < N; ++j) M[i * N + j] -= f * M[k * N + j];
      b[i] -= f * b[k];
    }
  }
  for (int32_t k = N - 1; k >= 0; --k) {
    double acc = b[k];
    for (int32_t j = k + 1; j < N; ++j) acc -= M[k * N + j] * x[j];
    x[k] = acc / M[k * N + k];
  }
  return 0;
}

/* Damping factor of the Newton-Raphson scheme at iteration it (Sec. 2.2):
 * 0.95, then 0.75, 0.5, 0.25 and 0.05 after 10, 35, 50 and 90 iterations. */
static double newton_damping(int it) {
  if (it < 10) return 0.95;
  if (it < 35) return 0.75;
  if (it < 50) return 0.5;
  if (it < 90) return 0.25;
  return 0.05;
}

/* The solve starts with at most FIXED_POINT_START_ITER fixed-point steps, until
 * the root-test residual is below FIXED_POINT_START_EXIT: from a start far from
 * the root (populations off by many decades) they close the distance at the
 * cost of one stationary vector each. Newton-Raphson steps are then limited
 * to change no level by more than a factor of 10 (NEWTON_MAX_LOG_STEP): the
 * paper limits the change of the populations between steps without giving
 * the limit; NEWTON_HALVINGS bounds the step halvings of one iteration. */
#define FIXED_POINT_START_ITER 30
#define FIXED_POINT_START_EXIT 0.1
#define NEWTON_MAX_LOG_STEP 2.302585092994046
#define NEWTON_HALVINGS 30
#define JACOBIAN_STEP 1e-5
/* The paper's convergence criterion: every level within 1 % of the fixed-point
 * map. The damping schedule serves the iteration up to that point; beyond it
 * (the oracle continues to tol) Newton steps are taken whole. */
#define PAPER_CONVERGENCE 0.01

/* The fixed-point map P(n) = n_tot * stationary(R(n)), the stationary
 * vector by GTH (oracle_gth), with the rates R(n) = R0 + decay(n) formed from
 * the population-independent rates R0 (rates_without_decay). Returns -1 if
 * it does not exist. */
static int fixed_point_map(const or_atom* a, const or_cells* cl, int32_t s, int32_t Ns,
                           double ntot, const double* R0, const double* n, double* R, double* P) {
  memcpy(R, R0, sizeof(double) * (size_t)Ns * Ns);
  add_decay(a, cl, s, n, R);
  oracle_gth(Ns, R, P);
  if (!(P[0] == P[0])) return -1;
  for (int32_t i = 0; i < Ns; ++i) P[i] *= ntot;
  return 0;
}

/* The equations in fixed-point form at y = ln n: H_i(y) = ln P(n)_i - y_i.
 * H = 0 exactly at the root. n and P are work arrays; returns -1 if P(n)
 * does not exist. */
static int equations(const or_atom* a, const or_cells* cl, int32_t s, int32_t Ns, double ntot,
                     const double* R0, const double* y, double* R, double* n, double* P,
                     double* H) {
  for (int32_t i = 0; i < Ns; ++i) n[i] = exp(y[i]);
  if (fixed_point_map(a, cl, s, Ns, ntot, R0, n, R, P) != 0) return -1;
  for (int32_t i = 0; i < Ns; ++i) H[i] = log(P[i]) - y[i];
  return 0;
}

/* Root-test residual max_i |P(n)_i / n_i - 1| from H = ln(P / n). */
static double root_residual(int32_t N, const double* H) {
  double r = 0.0;
  for (int32_t i = 0; i < N; ++i) if (fabs(expm1(H[i])) > r) r = fabs(expm1(H[i]));
  return r;
}

/* One species of one cell. n (local numbering, length Ns) holds the start on
 * entry and the solution on exit. Returns the number of iterations, or -1 if
 * the root test was not met within max_iter.
 *
 * The root is the fixed point of P(n) = n_tot * stationary(R(n)): the
 * stationary vector of the rates at n balances inflow and outflow of every
 * level, so n = P(n) is exactly the statistical equilibrium. P is computed
 * by GTH, which is subtraction-free and accurate for every component however
 * small.
 * 1. Fixed-point steps n <- P(n), damped in log(n) (w halved, down to 1/64,
 *    whenever the residual does not shrink), while far from the root.
 * 2. Newton-Raphson (Sec. 2.2: a numerical Jacobian built from a matrix
 *    calculation of all rates between all levels; a decreasing damping
 *    schedule) on H(y) = ln P(e^y) - y in y = ln n, so that populations stay
 *    positive. Jacobian column j is the central difference of H over
 *    y_j +- 1e-5; the correction d solves J d = -H by Gaussian elimination
 *    with partial pivoting. The step y + damp d takes damp from the paper's
 *    schedule (1 once max |H| is below the paper's 1 % criterion), lowered so
 *    that no level changes by more than a factor of 10, and halved until the
 *    residual max |H| decreases.
 * Stops only on the root test max_i |P(n)_i / n_i - 1| < tol. */
static int solve_species(const or_atom* a, const or_cells* cl, int64_t c, int32_t s, double* n,
                         int max_iter, double tol) {
  int32_t Ns = a->species_offset[s + 1] - a->species_offset[s];
  double ntot = cl->n_species[c * a->n_species + s];
  size_t NN = (size_t)Ns * Ns;
  double* R0 = (double*)malloc(sizeof(double) * NN);
  double* R = (double*)malloc(sizeof(double) * NN);
  double* J = (double*)malloc(sizeof(double) * NN);
  double* y = (double*)malloc(sizeof(double) * Ns);
  double* yt = (double*)malloc(sizeof(double) * Ns);
  double* H = (double*)malloc(sizeof(double) * Ns);
  double* Ht = (double*)malloc(sizeof(double) * Ns);
  double* d = (double*)malloc(sizeof(double) * Ns);
  double* P = (double*)malloc(sizeof(double) * Ns);
  double* work = (double*)malloc(sizeof(double) * Ns);
  int it = 0, result = -1;

  rates_without_decay(a, cl, c, s, R0);
  /* 1. damped fixed point while far from the root */
  double w = 1.0, prev = INFINITY;
  for (int k = 0; k < FIXED_POINT_START_ITER && it < max_iter; ++k) {
    if (fixed_point_map(a, cl, s, Ns, ntot, R0, n, R, P) != 0) goto done;
    double res = 0.0, sum = 0.0;
    for (int32_t i = 0; i < Ns; ++i)
      if (fabs(P[i] / n[i] - 1.0) > res) res = fabs(P[i] / n[i] - 1.0);
    if (res < FIXED_POINT_START_EXIT) break;
    ++it;
    if (res >= prev && w > 1.0 / 64) w *= 0.5;
    prev = res;
    for (int32_t i = 0; i < Ns; ++i) {
      n[i] = exp((1.0 - w) * log(n[i]) + w * log(P[i]));
      sum += n[i];
    }
    for (int32_t i = 0; i < Ns; ++i) n[i] *= ntot / sum;
  }

  /* 2. damped Newton-Raphson with a numerical Jacobian */
  for (int32_t i = 0; i < Ns; ++i) y[i] = log(n[i]);
  if (equations(a, cl, s, Ns, ntot, R0, y, R, work, P, H) != 0) goto done;
  for (int k = 0; it < max_iter; ++k) {
    double res = root_residual(Ns, H);
    if (res < tol) { result = it; break; }
    ++it;
    for (int32_t j = 0; j < Ns; ++j) {
      for (int32_t i = 0; i < Ns; ++i) yt[i] = y[i];
      yt[j] = y[j] + JACOBIAN_STEP;
      if (equations(a, cl, s, Ns, ntot, R0, yt, R, work, P, Ht) != 0) goto done;
      for (int32_t i = 0; i < Ns; ++i) J[i * Ns + j] = Ht[i];
      yt[j] = y[j] - JACOBIAN_STEP;
      if (equations(a, cl, s, Ns, ntot, R0, yt, R, work, P, Ht) != 0) goto done;
      for (int32_t i = 0; i < Ns; ++i) J[i * Ns + j] = (J[i * Ns + j] - Ht[i]) / (2.0 * JACOBIAN_STEP);
    }
    for (int32_t i = 0; i < Ns; ++i) Ht[i] = -H[i];
    if (gauss_solve(Ns, J, Ht, d) != 0) goto done;
    double big = 0.0;
    for (int32_t i = 0; i < Ns; ++i) if (fabs(d[i]) > big) big = fabs(d[i]);
    if (!(big < INFINITY)) goto done;
    double hmax = 0.0;
    for (int32_t i = 0; i < Ns; ++i) if (fabs(H[i]) > hmax) hmax = fabs(H[i]);
    double damp = hmax < PAPER_CONVERGENCE ? 1.0 : newton_damping(k);
    if (damp * big > NEWTON_MAX_LOG_STEP) damp = NEWTON_MAX_LOG_STEP / big;
    int accepted = 0;
    for (int h = 0; h < NEWTON_HALVINGS && !accepted; ++h, damp *= 0.5) {
      for (int32_t i = 0; i < Ns; ++i) yt[i] = y[i] + damp * d[i];
      if (equations(a, cl, s, Ns, ntot, R0, yt, R, work, P, Ht) != 0) continue;
      double tmax = 0.0;
      for (int32_t i = 0; i < Ns; ++i) if (fabs(Ht[i]) > tmax) tmax = fabs(Ht[i]);
      if (tmax < hmax) {
        accepted = 1;
        for (int32_t i = 0; i < Ns; ++i) { y[i] = yt[i]; H[i] = Ht[i]; }
      }
    }
    if (!accepted) break;
  }
  for (int32_t i = 0; i < Ns; ++i) n[i] = exp(y[i]);
done:
  free(R0); free(R); free(J); free(y); free(yt); free(H); free(Ht); free(d); free(P); free(work);
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
    if (max_iter <= 0) {  /* no iterations: the start is returned, not converged */
      status[c] = 2;
      if (iters) iters[c] = 0;
      continue;
    }
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
