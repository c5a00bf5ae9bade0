/* Oracle: Monte Carlo photon-packet transport with Sobolev line absorption.
 * Test infrastructure only (see oracle.h). FP64 throughout, one packet at a time.
 *
 * Physics, as the paper states it for its ray tracer (Sec. 2.3 "Radiative
 * transfer" and Sec. 2.3.2 "Photoexcitation"):
 *  - homologous flow: position in units of c*t equals velocity x = v/c;
 *  - at each step the ray's wavelength is moved to the comoving frame; the
 *    single next line redward of the current comoving wavelength is tested,
 *    and only lines with tau > 1e-4 in the current cell interact;
 *  - an interacting line absorbs N_phot*(1 - e^-tau) photons; the estimator
 *    receives that count divided by the stimulated-emission correction;
 *  - the ray stops when its remaining energy drops below 1e-6 of its start;
 *    rays that leave the grid escape.
 * Readings where the paper is silent:
 *  - first-order Doppler, lab frequency constant along a ray (rays never
 *    scatter): nu_cmf = nu_lab*(1 - n.x). With D = n.x, D grows by exactly
 *    the path length s, and line k resonates at D_k = 1 - lambda_lab/lambda_k;
 *  - per cell, lines with D_k in (D, D_exit] are processed in wavelength order;
 *    the line pointer starts at the first line with lambda_k > lambda_emit;
 *  - the kill test compares comoving energies: w*lambda_e < 1e-6*w0*lambda_k;
 *  - axes whose wall distances tie exactly are stepped together;
 *  - the packet's position on the crossed wall is set exactly to that wall.
 * Photoionisation (Sec. 2.3.1): every move of the ray -- to a wall, or to a
 * line that interacts -- also passes through the continuum of the
 * photoionising levels. Level i absorbs while the comoving wavelength is below
 * its threshold (the move is cut where the ray redshifts past it), with
 * tau_i = integral of sigma_i(lambda) n_i ds over that part; the move absorbs
 * N (1 - e^-tau), tau = sum_i tau_i, shared among the levels in proportion to
 * tau_i. Readings: sigma_i follows the ray's comoving wavelength along the
 * move (Eq. A5's lambda^3 law integrated exactly), and after a move that ends
 * at a wall the packet also stops once its comoving energy is below 1e-6 of
 * its start (the rule the paper states for the ray as a whole).
 * Emission (sampled mode): cell c emits cell_packets[c] packets with ids in
 * cell-major order; packet id p draws two Philox4x64-10 blocks with counters
 * (p, iteration, 0, 0) and (p, iteration, 1, 0) under key (seed, 3): uniform
 * position in the cell, isotropic direction, and a wavelength in stratum j of
 * n_c equal strata of [lambda_lo, lambda_hi]; weight cell_photons/n_c.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#include "oracle.h"

#define TAU_MIN 1e-4   /* Sec. 2.3.2: lines with tau_line > 1e-4 interact */
#define KILL_FRAC 1e-6 /* Sec. 2.3: ray followed until < 1e-6 of its energy remains */

typedef struct {
  or_record* r;
  int64_t n, cap;
} recbuf;

static void rec_push(recbuf* b, int64_t p, int32_t c, int32_t k, double v, double margin) {
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 1024;
    b->r = (or_record*)realloc(b->r, (size_t)b->cap * sizeof(or_record));
  }
  b->r[b->n].packet = p;
  b->r[b->n].cell = c;
  b->r[b->n].line = k;
  b->r[b->n].value = v;
  b->r[b->n].margin = margin;
  b->n++;
}

static double unit53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* lower wall coordinate of cell index i along one axis */
static double wall(const or_transport* P, int32_t i) {
  double h = 2.0 * P->beta_max / P->n;
  return -P->beta_max + (double)i * h;
}

static void line_tau(const or_transport* P, int64_t c, int32_t k, double* tau, double* fcorr) {
  if (P->line_trans && P->tau_ct && P->line_trans[k] >= 0) {
    int64_t t = P->line_trans[k];
    *tau = P->tau_ct[c * P->n_trans + t];
    *fcorr = P->fcorr_ct ? P->fcorr_ct[c * P->n_trans + t] : 1.0;
  } else {
    *tau = (double)P->line_tau0[k] * (double)P->tau_scale[c];
    *fcorr = 1.0;
  }
}

/* index of the first line with lambda > lam (upper bound) */
static int32_t first_line_above(const or_transport* P, double lam) {
  int32_t lo = 0, hi = P->n_lines;
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if (P->line_lambda[mid] > lam) hi = mid; else lo = mid + 1;
  }
  return lo;
}

typedef struct {
  int32_t ci[3];
  double x[3], dir[3], lam_e, w0;
} packet0;

static void emit_sampled(const or_transport* P, const int64_t* start, int64_t C, int64_t p,
                         packet0* q) {
  /* largest c with start[c] <= p; cells with no packets are skipped naturally */
  int64_t lo = 0, hi = C;
  while (hi - lo > 1) {
    int64_t mid = lo + (hi - lo) / 2;
    if (start[mid] <= p) lo = mid; else hi = mid;
  }
  int64_t c = lo;
  int64_t j = p - start[c];
  int32_t nc = P->cell_packets[c];
  int32_t n = P->n;
  q->ci[0] = (int32_t)(c % n);
  q->ci[1] = (int32_t)((c / n) % n);
  q->ci[2] = (int32_t)(c / ((int64_t)n * n));
  uint64_t key[2] = {P->seed, 3};
  uint64_t c0[4] = {(uint64_t)p, (uint64_t)(uint32_t)P->iteration, 0, 0};
  uint64_t c1[4] = {(uint64_t)p, (uint64_t)(uint32_t)P->iteration, 1, 0};
  uint64_t r0[4], r1[4];
  oracle_philox4x64(c0, key, r0);
  oracle_philox4x64(c1, key, r1);
  double h = 2.0 * P->beta_max / n;
  for (int a = 0; a < 3; ++a) q->x[a] = wall(P, q->ci[a]) + h * unit53(r0[a]);
  double mu = 2.0 * unit53(r0[3]) - 1.0;
  double phi = 2.0 * M_PI * unit53(r1[0]);
  double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  q->dir[0] = st * cos(phi);
  q->dir[1] = st * sin(phi);
  q->dir[2] = mu;
  q->lam_e = P->lambda_lo + (P->lambda_hi - P->lambda_lo) * (((double)j + unit53(r1[1])) / nc);
  q->w0 = P->cell_photons[c] / nc;
}

static void emit_explicit(const or_transport* P, int64_t p, packet0* q) {
  const double* e = P->explicit_packets + 8 * p;
  double h = 2.0 * P->beta_max / P->n;
  for (int a = 0; a < 3; ++a) {
    q->x[a] = e[a];
    q->dir[a] = e[3 + a];
    int32_t i = (int32_t)floor((e[a] + P->beta_max) / h);
    if (i < 0) i = 0;
    if (i > P->n - 1) i = P->n - 1;
    q->ci[a] = i;
  }
  q->lam_e = e[6];
  q->w0 = e[7];
}

/* Integral of lambda(D)^3 dD from D_a to D_b, lambda(D) = lambda_L / (1 - D),
 * given lambda_a = lambda(D_a), lambda_b = lambda(D_b): the antiderivative
 * lambda_L^3 / (2 (1 - D)^2) differenced, written as
 * (1/2) lambda_a lambda_b (lambda_a + lambda_b) (D_b - D_a), which has no
 * cancellation for short moves. */
static double lambda_cubed_integral(double lam_a, double lam_b, double dD) {
  return 0.5 * lam_a * lam_b * (lam_a + lam_b) * dD;
}

/* Photoionisation over the move D_a -> D_b of the ray in cell c with w
 * photons: returns the move's optical depth tau, sets *absorbed to
 * w (1 - e^-tau) and adds each level's share to pi_absorbed. */
static double photoionise(const or_transport* P, int64_t c, double lamL, double Da, double Db,
                          double w, double* absorbed) {
  *absorbed = 0.0;
  if (P->pi_levels <= 0 || !(Db > Da)) return 0.0;
  const int32_t M = P->pi_levels;
  double tau_i[M];
  double tau = 0.0;
  const double lam_a = lamL / (1.0 - Da);
  for (int32_t i = 0; i < M; ++i) {
    tau_i[i] = 0.0;
    const double lam_t = P->pi_lambda[i];
    if (!(lam_a < lam_t)) continue; /* already redward of the threshold */
    const double Dt = 1.0 - lamL / lam_t; /* where the ray reaches the threshold */
    double lam_b, dD;
    if (Dt < Db) { lam_b = lam_t; dD = Dt - Da; }
    else { lam_b = lamL / (1.0 - Db); dD = Db - Da; }
    const double n_i = P->pi_pops[c * P->pi_nlev + P->pi_level[i]];
    const double k = n_i * P->pi_sigma0[i] / (lam_t * lam_t * lam_t);
    tau_i[i] = k * lambda_cubed_integral(lam_a, lam_b, dD) * P->pi_length;
    tau += tau_i[i];
  }
  if (!(tau > 0.0)) return 0.0;
  const double N = w * (-expm1(-tau));
  for (int32_t i = 0; i < M; ++i)
    if (tau_i[i] > 0.0) P->pi_absorbed[c * M + i] += N * (tau_i[i] / tau);
  *absorbed = N;
  return tau;
}

/* Follows one packet; returns nothing, fills out[12], stats, records. */
static void follow(const or_transport* P, int64_t p, const packet0* q, recbuf* rb, double* st,
                   double* out) {
  int32_t n = P->n;
  int32_t ci[3] = {q->ci[0], q->ci[1], q->ci[2]};
  double x[3] = {q->x[0], q->x[1], q->x[2]};
  const double* dir = q->dir;
  double D = dir[0] * x[0] + dir[1] * x[1] + dir[2] * x[2];
  double lamL = q->lam_e * (1.0 - D);         /* lab wavelength, fixed along the ray */
  int32_t k = first_line_above(P, q->lam_e);  /* no absorption at the emission wavelength */
  double h = 2.0 * P->beta_max / n;
  double w = q->w0, Dcur = D;
  double e_abs = 0.0, e_adiab = 0.0, w_abs = 0.0, w_pi = 0.0;
  double res[OR_PKT_FIELDS] = {0};
  res[1] = lamL;
  res[6] = q->w0 / q->lam_e;
  st[0] += q->w0;
  for (;;) {
    int64_t c = ci[0] + (int64_t)n * (ci[1] + (int64_t)n * ci[2]);
    double dist[3], smin = INFINITY;
    for (int a = 0; a < 3; ++a) {
      dist[a] = INFINITY;
      if (dir[a] > 0.0) dist[a] = (wall(P, ci[a] + 1) - x[a]) / dir[a];
      else if (dir[a] < 0.0) dist[a] = (wall(P, ci[a]) - x[a]) / dir[a];
      if (dist[a] < smin) smin = dist[a];
    }
    double s = smin > 0.0 ? smin : 0.0;
    double Dexit = D + s;
    while (k < P->n_lines) {
      double lamk = P->line_lambda[k];
      double Dk = 1.0 - lamL / lamk;
      if (Dk > Dexit) break;
      st[5] += 1.0;
      double tau, fcorr;
      line_tau(P, c, k, &tau, &fcorr);
      if (tau > TAU_MIN) {
        st[4] += 1.0;
        e_adiab += w * (Dk - Dcur) / lamL;
        if (P->pi_levels > 0) {
          double Npi;
          const double tpi = photoionise(P, c, lamL, Dcur, Dk, w, &Npi);
          if (tpi > 0.0) {
            w_pi += Npi;
            w = w * exp(-tpi);
          }
        }
        Dcur = Dk;
        double dN = w * (-expm1(-tau));
        double m1 = Dk - D, m2 = Dexit - Dk;
        rec_push(rb, p, (int32_t)c, k, dN / fcorr, (m1 < m2 ? m1 : m2) / h);
        w_abs += dN;
        e_abs += dN / lamk;
        w = w * exp(-tau);  /* N_phot - N_PE = N_phot e^-tau, in the accurate form */
        if (w * q->lam_e < (KILL_FRAC * q->w0) * lamk) {
          res[2] = w;
          res[7] = w / lamk;
          st[2] += w;
          st[8] += 1.0;
          goto done;
        }
      }
      ++k;
    }
    e_adiab += w * (Dexit - Dcur) / lamL;
    if (P->pi_levels > 0) {
      double Npi;
      const double tpi = photoionise(P, c, lamL, Dcur, Dexit, w, &Npi);
      if (tpi > 0.0) {
        w_pi += Npi;
        w = w * exp(-tpi);
        /* comoving energy left at the wall against 1e-6 of the start */
        if (w * q->lam_e * (1.0 - Dexit) < (KILL_FRAC * q->w0) * lamL) {
          res[2] = w;
          res[7] = w * (1.0 - Dexit) / lamL;
          st[2] += w;
          st[8] += 1.0;
          goto done;
        }
      }
    }
    Dcur = Dexit;
    D = Dexit;
    int out_of_grid = 0;
    for (int a = 0; a < 3; ++a) {
      if (dist[a] == smin) {
        if (dir[a] > 0.0) { ci[a] += 1; x[a] = wall(P, ci[a]); }
        else { x[a] = wall(P, ci[a]); ci[a] -= 1; }
        if (ci[a] < 0 || ci[a] >= n) out_of_grid = 1;
      } else {
        x[a] = x[a] + s * dir[a];
      }
    }
    if (out_of_grid) {
      res[0] = w;
      res[7] = w * (1.0 - D) / lamL;
      st[1] += w;
      st[7] += 1.0;
      goto done;
    }
    st[6] += 1.0;
  }
done:
  st[3] += w_abs;
  st[9] += w_pi;
  res[11] = w_pi;
  res[3] = w_abs;
  res[4] = e_abs;
  res[5] = e_adiab;
  res[8] = dir[0];
  res[9] = dir[1];
  res[10] = dir[2];
  if (out) memcpy(out, res, sizeof(res));
}

int64_t oracle_transport(const or_transport* P, int64_t first, int64_t count, int nthreads,
                         or_record** records, double* stats, double* pkt_out) {
  if (!P || P->n <= 0 || P->n_lines < 0 || count < 0) return -1;
  if (P->pi_levels > 0) {
    if (!P->pi_lambda || !P->pi_sigma0 || !P->pi_level || !P->pi_pops || !P->pi_absorbed)
      return -1;
    nthreads = 1; /* one absorption table, filled in packet order */
  }
  for (int32_t k = 1; k < P->n_lines; ++k)
    if (!(P->line_lambda[k] >= P->line_lambda[k - 1])) return -1;
  int64_t C = (int64_t)P->n * P->n * P->n;
  int64_t* start = NULL;
  if (!P->explicit_packets) {
    start = (int64_t*)malloc((size_t)(C + 1) * sizeof(int64_t));
    start[0] = 0;
    for (int64_t c = 0; c < C; ++c) start[c + 1] = start[c] + P->cell_packets[c];
    if (first + count > start[C]) { free(start); return -1; }
  }
  if (nthreads < 1) nthreads = 1;
  recbuf* bufs = (recbuf*)calloc((size_t)nthreads, sizeof(recbuf));
  double* tstats = (double*)calloc((size_t)nthreads * OR_STATS, sizeof(double));
#pragma omp parallel num_threads(nthreads)
  {
    int t = omp_get_thread_num();
    int nt = omp_get_num_threads();
    int64_t a = first + count * t / nt, b = first + count * (t + 1) / nt;
    for (int64_t p = a; p < b; ++p) {
      packet0 q;
      if (P->explicit_packets) emit_explicit(P, p, &q);
      else emit_sampled(P, start, C, p, &q);
      follow(P, p, &q, &bufs[t], tstats + OR_STATS * t,
             pkt_out ? pkt_out + OR_PKT_FIELDS * (p - first) : NULL);
    }
  }
  /* merge in thread order == packet order */
  int64_t total = 0;
  for (int t = 0; t < nthreads; ++t) total += bufs[t].n;
  or_record* all = (or_record*)malloc((size_t)(total > 0 ? total : 1) * sizeof(or_record));
  int64_t off = 0;
  for (int t = 0; t < nthreads; ++t) {
    if (bufs[t].n) memcpy(all + off, bufs[t].r, (size_t)bufs[t].n * sizeof(or_record));
    off += bufs[t].n;
    free(bufs[t].r);
  }
  if (stats) {
    for (int i = 0; i < OR_STATS; ++i) stats[i] = 0.0;
    for (int t = 0; t < nthreads; ++t)
      for (int i = 0; i < OR_STATS; ++i) stats[i] += tstats[OR_STATS * t + i];
  }
  free(tstats);
  free(bufs);
  free(start);
  *records = all;
  return total;
}

int oracle_emission(const or_transport* P, int64_t first, int64_t count, double* out) {
  if (!P || P->n <= 0 || count < 0 || first < 0) return -1;
  int64_t C = (int64_t)P->n * P->n * P->n;
  int64_t* start = NULL;
  if (!P->explicit_packets) {
    start = (int64_t*)malloc((size_t)(C + 1) * sizeof(int64_t));
    start[0] = 0;
    for (int64_t c = 0; c < C; ++c) start[c + 1] = start[c] + P->cell_packets[c];
    if (first + count > start[C]) { free(start); return -1; }
  }
  for (int64_t p = first; p < first + count; ++p) {
    packet0 q;
    if (P->explicit_packets) emit_explicit(P, p, &q);
    else emit_sampled(P, start, C, p, &q);
    double* o = out + 8 * (p - first);
    for (int a = 0; a < 3; ++a) { o[a] = q.x[a]; o[3 + a] = q.dir[a]; }
    o[6] = q.lam_e;
    o[7] = q.w0;
  }
  free(start);
  return 0;
}

void oracle_free(void* ptr) { free(ptr); }

/* Eq. A2: tau_S = (A_ul/8pi)(g_u/g_l) lambda^3 n_l (1 - g_l n_u/(g_u n_l)) t.
 * Also returns the stimulated-emission factor f_corr = 1 - g_l n_u/(g_u n_l),
 * the reading taken for the correction in the photoexcitation count. */
void oracle_line_tau(int64_t n_cells, int32_t n_levels, int32_t n_trans, const double* pops,
                     const int32_t* lower, const int32_t* upper, const double* A,
                     const double* lambda, const double* g, double t_exp,
                     double* tau_ct, double* fcorr_ct) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n_cells; ++c) {
    for (int32_t t = 0; t < n_trans; ++t) {
      double nl = pops[c * n_levels + lower[t]];
      double nu = pops[c * n_levels + upper[t]];
      double gl = g[lower[t]], gu = g[upper[t]];
      double tau = 0.0, fc = 1.0;
      if (nl > 0.0) {
        fc = 1.0 - (gl * nu) / (gu * nl);
        double lam = lambda[t];
        tau = A[t] / (8.0 * M_PI) * (gu / gl) * lam * lam * lam * nl * fc * t_exp;
      }
      tau_ct[c * n_trans + t] = tau;
      fcorr_ct[c * n_trans + t] = fc;
    }
  }
}

/* Sec. 2.3.1/2.3.2: absorbed photons per second in a line of a cell, divided
 * by the number of atoms in the lower level (population times cell volume),
 * give the photoexcitation rate per lower atom. */
void oracle_rates(int64_t n_cells, int32_t n_lines, int32_t n_levels, int32_t n_trans,
                  const double* est, const double* pops, const int32_t* lower,
                  const int32_t* trans_line, double cell_volume, double* gamma_pe) {
  for (int64_t c = 0; c < n_cells; ++c) {
    for (int32_t t = 0; t < n_trans; ++t) {
      double Nl = pops[c * n_levels + lower[t]] * cell_volume;
      double e = est[c * n_lines + trans_line[t]];
      gamma_pe[c * n_trans + t] = Nl > 0.0 ? e / Nl : 0.0;
    }
  }
}
