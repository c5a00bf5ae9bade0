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

/* Sampled emission in a spherical cell: r^3 uniform over the shell (u0),
 * cos(theta) uniform over the polar bin (u1), phi uniform over the slice
 * (u2), i.e. uniform in the cell's volume; the rest as in the cube. */
static void emit_sampled_sph(const or_transport* P, const int64_t* start, int64_t C, int64_t p,
                             packet0* q) {
  const or_sphere* g = P->sphere;
  int64_t lo = 0, hi = C;
  while (hi - lo > 1) {
    int64_t mid = lo + (hi - lo) / 2;
    if (start[mid] <= p) lo = mid; else hi = mid;
  }
  const int64_t c = lo;
  const int64_t j = p - start[c];
  const int32_t nc = P->cell_packets[c];
  const int32_t ir = (int32_t)(c % g->n_r);
  const int32_t it = (int32_t)((c / g->n_r) % g->n_theta);
  const int32_t ip = (int32_t)(c / ((int64_t)g->n_r * g->n_theta));
  q->ci[0] = ir; q->ci[1] = it; q->ci[2] = ip;
  uint64_t key[2] = {P->seed, 3};
  uint64_t c0[4] = {(uint64_t)p, (uint64_t)(uint32_t)P->iteration, 0, 0};
  uint64_t c1[4] = {(uint64_t)p, (uint64_t)(uint32_t)P->iteration, 1, 0};
  uint64_t r0[4], r1[4];
  oracle_philox4x64(c0, key, r0);
  oracle_philox4x64(c1, key, r1);
  const double ra = g->r_edge[ir], rb = g->r_edge[ir + 1];
  const double r = cbrt(ra * ra * ra + unit53(r0[0]) * (rb * rb * rb - ra * ra * ra));
  const double ca = cos(g->theta_edge[it]), cb = cos(g->theta_edge[it + 1]);
  const double mu_x = ca + unit53(r0[1]) * (cb - ca);
  const double ph_x = 2.0 * M_PI * (ip + unit53(r0[2])) / g->n_phi;
  const double sx = sqrt(fmax(0.0, 1.0 - mu_x * mu_x));
  q->x[0] = r * sx * cos(ph_x);
  q->x[1] = r * sx * sin(ph_x);
  q->x[2] = r * mu_x;
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
    q->ci[a] = 0;
    if (P->sphere) continue; /* the spherical follow finds the cell itself */
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

/* ---- spherical grid ------------------------------------------------------ */

static int64_t sphere_cells(const or_sphere* g) {
  return (int64_t)g->n_r * g->n_theta * g->n_phi;
}

/* last index i with e[i] <= v among e[0..n] (n + 1 edges), clamped to [0, n-1] */
static int32_t bin_of(const double* e, int32_t n, double v) {
  int32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) / 2;
    if (e[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

int64_t oracle_sphere_cell(const or_sphere* g, const double x[3]) {
  const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  if (!(r < g->r_edge[g->n_r])) return -1;
  const int32_t ir = bin_of(g->r_edge, g->n_r, r);
  double ct = r > 0.0 ? x[2] / r : 1.0;
  if (ct > 1.0) ct = 1.0;
  if (ct < -1.0) ct = -1.0;
  const int32_t it = bin_of(g->theta_edge, g->n_theta, acos(ct));
  double phi = atan2(x[1], x[0]);
  if (phi < 0.0) phi += 2.0 * M_PI;
  int32_t ip = (int32_t)floor(phi / (2.0 * M_PI / g->n_phi));
  if (ip < 0) ip = 0;
  if (ip > g->n_phi - 1) ip = g->n_phi - 1;
  return ir + (int64_t)g->n_r * (it + (int64_t)g->n_theta * ip);
}

static int cmp_double(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

static void push_root(double s, double* out, int32_t* m, int32_t cap) {
  if (s > 0.0 && *m < cap) out[(*m)++] = s;
}

int32_t oracle_sphere_crossings(const or_sphere* g, const double x0[3], const double n[3],
                                double* out, int32_t cap) {
  const double b = x0[0] * n[0] + x0[1] * n[1] + x0[2] * n[2];
  const double xx = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2];
  const double R = g->r_edge[g->n_r];
  const double discR = b * b - (xx - R * R);
  if (!(discR > 0.0)) return 0;
  const double s_end = -b + sqrt(discR); /* last exit from the outer sphere */
  int32_t m = 0;
  /* spheres |x0 + s n| = r */
  for (int32_t i = 1; i <= g->n_r; ++i) {
    const double r = g->r_edge[i];
    const double disc = b * b - (xx - r * r);
    if (disc < 0.0) continue;
    const double q = sqrt(disc);
    push_root(-b - q, out, &m, cap);
    push_root(-b + q, out, &m, cap);
  }
  /* cones theta = theta_j: z = cos(theta_j) |x| */
  for (int32_t j = 1; j < g->n_theta; ++j) {
    const double c = cos(g->theta_edge[j]);
    if (fabs(c) < 1e-15) { /* the equatorial plane */
      if (n[2] != 0.0) push_root(-x0[2] / n[2], out, &m, cap);
      continue;
    }
    const double A = n[2] * n[2] - c * c;
    const double B = x0[2] * n[2] - c * c * b;
    const double Cq = x0[2] * x0[2] - c * c * xx;
    double roots[2];
    int nr = 0;
    if (fabs(A) < 1e-300) {
      if (B != 0.0) roots[nr++] = -Cq / (2.0 * B);
    } else {
      const double disc = B * B - A * Cq;
      if (disc >= 0.0) {
        const double q = sqrt(disc);
        roots[nr++] = (-B - q) / A;
        roots[nr++] = (-B + q) / A;
      }
    }
    for (int k = 0; k < nr; ++k) {
      const double z = x0[2] + roots[k] * n[2];
      if ((z > 0.0) == (c > 0.0)) push_root(roots[k], out, &m, cap); /* the cone's own nappe */
    }
  }
  /* half-planes phi = phi_k through the z axis */
  if (g->n_phi > 1) {
    for (int32_t k = 0; k < g->n_phi; ++k) {
      const double ph = 2.0 * M_PI * k / g->n_phi;
      const double cp = cos(ph), sp = sin(ph);
      const double den = -sp * n[0] + cp * n[1];
      if (den == 0.0) continue;
      const double sr = (sp * x0[0] - cp * x0[1]) / den;
      const double px = x0[0] + sr * n[0], py = x0[1] + sr * n[1];
      if (cp * px + sp * py > 0.0) push_root(sr, out, &m, cap);
    }
  }
  int32_t k = 0;
  for (int32_t i = 0; i < m; ++i)
    if (out[i] < s_end) out[k++] = out[i];
  m = k;
  if (m < cap) out[m++] = s_end;
  qsort(out, (size_t)m, sizeof(double), cmp_double);
  return m;
}

/* State of a packet along its ray. */
typedef struct {
  double lamL;       /* lab wavelength, fixed along the ray */
  int32_t k;         /* next line to test */
  double w, Dcur;    /* photons left; D where the last absorption left the ray */
  double e_abs, e_adiab, w_abs, w_pi;
} raystate;

/* The lines and the continuum of one segment of the ray, D -> Dexit, inside
 * cell c (Sec. 2.3.1, 2.3.2). h scales the recorded margins (a cell width).
 * Returns 1 when the packet stops there (the 1e-6 rule), with res[2], res[7]
 * and the kill tallies set. */
static int segment(const or_transport* P, int64_t p, const packet0* q, int64_t c, double D,
                   double Dexit, double h, raystate* R, recbuf* rb, double* st, double* res) {
  const double lamL = R->lamL;
  while (R->k < P->n_lines) {
    double lamk = P->line_lambda[R->k];
    double Dk = 1.0 - lamL / lamk;
    if (Dk > Dexit) break;
    st[5] += 1.0;
    double tau, fcorr;
    line_tau(P, c, R->k, &tau, &fcorr);
    if (tau > TAU_MIN) {
      st[4] += 1.0;
      R->e_adiab += R->w * (Dk - R->Dcur) / lamL;
      if (P->pi_levels > 0) {
        double Npi;
        const double tpi = photoionise(P, c, lamL, R->Dcur, Dk, R->w, &Npi);
        if (tpi > 0.0) {
          R->w_pi += Npi;
          R->w = R->w * exp(-tpi);
        }
      }
      R->Dcur = Dk;
      double dN = R->w * (-expm1(-tau));
      double m1 = Dk - D, m2 = Dexit - Dk;
      rec_push(rb, p, (int32_t)c, R->k, dN / fcorr, (m1 < m2 ? m1 : m2) / h);
      R->w_abs += dN;
      R->e_abs += dN / lamk;
      R->w = R->w * exp(-tau);  /* N_phot - N_PE = N_phot e^-tau, in the accurate form */
      if (R->w * q->lam_e < (KILL_FRAC * q->w0) * lamk) {
        res[2] = R->w;
        res[7] = R->w / lamk;
        st[2] += R->w;
        st[8] += 1.0;
        return 1;
      }
    }
    ++R->k;
  }
  R->e_adiab += R->w * (Dexit - R->Dcur) / lamL;
  if (P->pi_levels > 0) {
    double Npi;
    const double tpi = photoionise(P, c, lamL, R->Dcur, Dexit, R->w, &Npi);
    if (tpi > 0.0) {
      R->w_pi += Npi;
      R->w = R->w * exp(-tpi);
      /* comoving energy left at the wall against 1e-6 of the start */
      if (R->w * q->lam_e * (1.0 - Dexit) < (KILL_FRAC * q->w0) * lamL) {
        res[2] = R->w;
        res[7] = R->w * (1.0 - Dexit) / lamL;
        st[2] += R->w;
        st[8] += 1.0;
        return 1;
      }
    }
  }
  R->Dcur = Dexit;
  return 0;
}

static void start_ray(const packet0* q, double D, raystate* R, double* st, double* res) {
  R->lamL = q->lam_e * (1.0 - D);
  R->w = q->w0;
  R->Dcur = D;
  R->e_abs = R->e_adiab = R->w_abs = R->w_pi = 0.0;
  res[1] = R->lamL;
  res[6] = q->w0 / q->lam_e;
  st[0] += q->w0;
}

static void finish_ray(const packet0* q, const raystate* R, double* st, double* res,
                       double* out) {
  st[3] += R->w_abs;
  st[9] += R->w_pi;
  res[11] = R->w_pi;
  res[3] = R->w_abs;
  res[4] = R->e_abs;
  res[5] = R->e_adiab;
  res[8] = q->dir[0];
  res[9] = q->dir[1];
  res[10] = q->dir[2];
  if (out) memcpy(out, res, OR_PKT_FIELDS * sizeof(double));
}

static void escape_ray(const raystate* R, double D, double* st, double* res) {
  res[0] = R->w;
  res[7] = R->w * (1.0 - D) / R->lamL;
  st[1] += R->w;
  st[7] += 1.0;
}

/* Follows one packet through the cube (cell walls, tied axes stepped
 * together); fills out[12], stats, records. */
static void follow(const or_transport* P, int64_t p, const packet0* q, recbuf* rb, double* st,
                   double* out) {
  int32_t n = P->n;
  int32_t ci[3] = {q->ci[0], q->ci[1], q->ci[2]};
  double x[3] = {q->x[0], q->x[1], q->x[2]};
  const double* dir = q->dir;
  double D = dir[0] * x[0] + dir[1] * x[1] + dir[2] * x[2];
  double h = 2.0 * P->beta_max / n;
  double res[OR_PKT_FIELDS] = {0};
  raystate R;
  start_ray(q, D, &R, st, res);
  R.k = first_line_above(P, q->lam_e);  /* no absorption at the emission wavelength */
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
    if (segment(P, p, q, c, D, Dexit, h, &R, rb, st, res)) break;
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
      escape_ray(&R, D, st, res);
      break;
    }
    st[6] += 1.0;
  }
  finish_ray(q, &R, st, res, out);
}

/* Follows one packet through the spherical grid: the ray is cut at every
 * crossing of a grid surface, each piece lies in the cell its midpoint falls
 * in (consecutive pieces in one cell, where the ray only touches a surface,
 * form one segment); fills out[12], stats, records. */
static void follow_sph(const or_transport* P, int64_t p, const packet0* q, recbuf* rb,
                       double* st, double* out) {
  const or_sphere* g = P->sphere;
  const double* dir = q->dir;
  const double D0 = dir[0] * q->x[0] + dir[1] * q->x[1] + dir[2] * q->x[2];
  const double h = g->r_edge[g->n_r] / g->n_r;
  double res[OR_PKT_FIELDS] = {0};
  raystate R;
  start_ray(q, D0, &R, st, res);
  R.k = first_line_above(P, q->lam_e);
  const int32_t cap = 2 * g->n_r + 2 * g->n_theta + g->n_phi + 4;
  double* cut = (double*)malloc((size_t)cap * sizeof(double));
  const int32_t m = oracle_sphere_crossings(g, q->x, dir, cut, cap);
  double s_a = 0.0, D = D0;
  int64_t c = -1;
  int stopped = 0;
  for (int32_t i = 0; i < m && !stopped; ++i) {
    const double s_b = cut[i];
    if (!(s_b > s_a)) continue;
    const double sm = 0.5 * (s_a + s_b);
    const double xm[3] = {q->x[0] + sm * dir[0], q->x[1] + sm * dir[1], q->x[2] + sm * dir[2]};
    const int64_t cm = oracle_sphere_cell(g, xm);
    /* the segment in cell c ends where the next piece lies in another cell;
     * a ray that starts outside the grid begins where it enters */
    if (cm != c) {
      if (c >= 0) {
        const double Dexit = D0 + s_a;
        stopped = segment(P, p, q, c, D, Dexit, h, &R, rb, st, res);
        D = Dexit;
        if (!stopped && cm >= 0) st[6] += 1.0;
      } else {
        D = D0 + s_a;
        R.Dcur = D;
      }
    }
    c = cm;
    s_a = s_b;
  }
  if (!stopped && c >= 0) {
    const double Dexit = D0 + s_a;
    stopped = segment(P, p, q, c, D, Dexit, h, &R, rb, st, res);
    D = Dexit;
  }
  if (!stopped) escape_ray(&R, D, st, res);
  free(cut);
  finish_ray(q, &R, st, res, out);
}

int64_t oracle_transport(const or_transport* P, int64_t first, int64_t count, int nthreads,
                         or_record** records, double* stats, double* pkt_out) {
  if (!P || (!P->sphere && P->n <= 0) || P->n_lines < 0 || count < 0) return -1;
  if (P->pi_levels > 0) {
    if (!P->pi_lambda || !P->pi_sigma0 || !P->pi_level || !P->pi_pops || !P->pi_absorbed)
      return -1;
    nthreads = 1; /* one absorption table, filled in packet order */
  }
  for (int32_t k = 1; k < P->n_lines; ++k)
    if (!(P->line_lambda[k] >= P->line_lambda[k - 1])) return -1;
  if (P->sphere && (P->sphere->n_r < 1 || P->sphere->n_theta < 1 || P->sphere->n_phi < 1))
    return -1;
  int64_t C = P->sphere ? sphere_cells(P->sphere) : (int64_t)P->n * P->n * P->n;
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
      else if (P->sphere) emit_sampled_sph(P, start, C, p, &q);
      else emit_sampled(P, start, C, p, &q);
      double* po = pkt_out ? pkt_out + OR_PKT_FIELDS * (p - first) : NULL;
      if (P->sphere) follow_sph(P, p, &q, &bufs[t], tstats + OR_STATS * t, po);
      else follow(P, p, &q, &bufs[t], tstats + OR_STATS * t, po);
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
  if (!P || (!P->sphere && P->n <= 0) || count < 0 || first < 0) return -1;
  int64_t C = P->sphere ? sphere_cells(P->sphere) : (int64_t)P->n * P->n * P->n;
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
    else if (P->sphere) emit_sampled_sph(P, start, C, p, &q);
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
                  const int32_t* trans_line, double cell_volume, const double* volumes,
                  double* gamma_pe) {
  for (int64_t c = 0; c < n_cells; ++c) {
    const double V = volumes ? volumes[c] : cell_volume;
    for (int32_t t = 0; t < n_trans; ++t) {
      double Nl = pops[c * n_levels + lower[t]] * V;
      double e = est[c * n_lines + trans_line[t]];
      gamma_pe[c * n_trans + t] = Nl > 0.0 ? e / Nl : 0.0;
    }
  }
}
