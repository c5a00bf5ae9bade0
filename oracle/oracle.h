/* Plain FP64 CPU oracle for the ExTraSS hot path (arXiv 2511.07539).
 *
 * TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load it. The product path (the HIP library)
 * never links, calls or falls back to this code, and the two share no source.
 *
 * Everything here is FP64, serial per packet / per cell, written for
 * readability rather than speed. Each function cites the passage of the paper
 * it follows. Where the paper is silent, the reading taken is stated at the
 * function.
 */
#ifndef EXTRASS_ORACLE_H
#define EXTRASS_ORACLE_H
#include <stdint.h>

/* ---- Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11) ------------------ */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* ---- Transport --------------------------------------------------------------
 * Grid: cube [-beta_max, beta_max]^3 in x = v/c with n cells per axis,
 * cell c = i + n*(j + n*k). Lines sorted by rest wavelength (cm).
 * tau(c,k) = line_tau0[k]*tau_scale[c] for background lines (line_trans[k] < 0
 * or line_trans == NULL); tau_ct[c*n_trans + t] for line k = transition t.
 */
/* Spherical grid (the paper's (r, theta, phi) cells, Sec. 2): n_r shells with
 * edges r_edge[0] = 0 < ... < r_edge[n_r] in x = v/c, n_theta polar bins with
 * edges theta_edge[0] = 0 < ... < theta_edge[n_theta] = pi, n_phi equal
 * azimuthal slices of 2 pi / n_phi starting at phi = 0. Cell
 * c = i_r + n_r (i_theta + n_theta i_phi): a phi slice is a contiguous range. */
typedef struct {
  int32_t n_r, n_theta, n_phi;
  const double* r_edge;         /* [n_r + 1] */
  const double* theta_edge;     /* [n_theta + 1] */
} or_sphere;

typedef struct {
  int32_t n;
  double beta_max;
  const float* tau_scale;       /* [C] */
  const double* cell_photons;   /* [C] photons s^-1 */
  const int32_t* cell_packets;  /* [C] packets per cell */
  int32_t n_lines;
  const double* line_lambda;    /* [L] cm ascending */
  const float* line_tau0;       /* [L] */
  const int32_t* line_trans;    /* [L] or NULL */
  int32_t n_trans;
  const double* tau_ct;         /* [C*T] or NULL */
  const double* fcorr_ct;       /* [C*T] or NULL */
  double lambda_lo, lambda_hi;  /* emission band, cm */
  uint64_t seed;
  int32_t iteration;
  const double* explicit_packets; /* [P*8] x,y,z,nx,ny,nz,lambda_e,w0; NULL = sampled */
  /* Photoionisation (Sec. 2.3.1; Eq. A5), or pi_levels = 0. Level i (of
   * oracle_pi_levels) with threshold pi_lambda[i] and threshold cross section
   * pi_sigma0[i] absorbs along every move of the ray while the comoving
   * wavelength is below its threshold, with population pi_pops[c*pi_nlev +
   * pi_level[i]] (cm^-3). pi_absorbed [C*M] accumulates the photons each level
   * absorbs in each cell; it needs nthreads == 1 (one table, packet order). */
  int32_t pi_levels;
  const double* pi_lambda;        /* [M] cm */
  const double* pi_sigma0;        /* [M] cm^2 */
  const int32_t* pi_level;        /* [M] */
  int32_t pi_nlev;
  const double* pi_pops;          /* [C*pi_nlev] */
  double pi_length;               /* cm per unit of path, c t_exp */
  double* pi_absorbed;            /* [C*M] out, accumulated */
  /* Spherical grid instead of the cube (n and beta_max unused), or NULL.
   * Sampled emission in cell (i_r, i_theta, i_phi) takes r^3 uniform in the
   * shell (u0), cos(theta) uniform in the polar bin (u1) and phi uniform in
   * the slice (u2); direction, wavelength and weight as in the cube. The
   * path is cut at every crossing of a sphere, cone or half-plane of the
   * grid; each piece lies in the cell its midpoint falls in. */
  const or_sphere* sphere;
} or_transport;

/* Per-packet results (12 doubles per packet):
 * 0 escaped weight, 1 lab wavelength lambda_L, 2 killed weight,
 * 3 photons absorbed in lines (sum of dN), 4 comoving energy / (hc) absorbed
 * in lines, 5 adiabatic loss / (hc), 6 emitted comoving energy / (hc),
 * 7 remaining comoving energy / (hc) at escape or kill,
 * 8-10 lab-frame direction (unchanged along the ray),
 * 11 photons absorbed by photoionisation. */
enum { OR_PKT_FIELDS = 12 };
/* Global stats (doubles): w_emit, w_esc, w_kill, w_abs, n_inter, n_checks,
 * n_cross, n_escaped, n_killed, w_pi (photons absorbed by photoionisation). */
enum { OR_STATS = 10 };

/* One line interaction: packet, cell, line, photons added to est (dN / f_corr),
 * and the margin of the resonance inside its segment, min(D_k - D_entry,
 * D_exit - D_k) / h (how far the decision "this line, this cell" was from a
 * wall; used to classify reduced-precision differences as near ties). */
typedef struct { int64_t packet; int32_t cell, line; double value, margin; } or_record;

/* Runs packets [first, first+count). Returns the number of records written to
 * *records (malloc'ed; free with oracle_free), or -1 on invalid input. */
int64_t oracle_transport(const or_transport* p, int64_t first, int64_t count, int nthreads,
                         or_record** records, double* stats, double* pkt_out);
void oracle_free(void* ptr);

/* Cell of point x on a spherical grid, -1 outside (exposed for the pins). */
int64_t oracle_sphere_cell(const or_sphere* g, const double x[3]);
/* Path lengths s > 0 (ascending, at most cap) at which the ray x0 + s n meets
 * a surface of the spherical grid, up to its last exit from the outer sphere.
 * Returns how many (exposed for the pins). */
int32_t oracle_sphere_crossings(const or_sphere* g, const double x0[3], const double n[3],
                                double* s_out, int32_t cap);

/* The emitted state of packets [first, first+count), as the transport draws
 * it: out[8*i .. 8*i+7] = x, y, z, n_x, n_y, n_z, lambda_e, w0 (the layout of
 * an explicit packet). Returns -1 on invalid input. Exposed for the pins. */
int oracle_emission(const or_transport* p, int64_t first, int64_t count, double* out);

/* ---- Eq. A2 line optical depth from populations --------------------------- */
void oracle_line_tau(int64_t n_cells, int32_t n_levels, int32_t n_trans, const double* pops,
                     const int32_t* lower, const int32_t* upper, const double* A,
                     const double* lambda, const double* g, double t_exp,
                     double* tau_ct, double* fcorr_ct);

/* ---- Photoexcitation rates -------------------------------------------------- */
/* V is volumes[c] (cm^3, per cell, a spherical grid's) when volumes is not
 * NULL, else cell_volume. */
void oracle_rates(int64_t n_cells, int32_t n_lines, int32_t n_levels, int32_t n_trans,
                  const double* est, const double* pops, const int32_t* lower,
                  const int32_t* trans_line, double cell_volume, const double* volumes,
                  double* gamma_pe);

/* ---- NLTE statistical equilibrium ------------------------------------------ */
typedef struct {
  int32_t n_species;
  const int32_t* species_offset;  /* [S+1] */
  int32_t n_levels;
  const int32_t* level_ion;       /* [N] */
  const double* level_energy;     /* [N] erg */
  const double* level_g;          /* [N] */
  int32_t n_trans;
  const int32_t* trans_lower, *trans_upper;  /* [T] */
  const double* trans_A, *trans_lambda, *trans_upsilon;  /* [T] */
  const double* ion_alpha0;       /* [S*3] cm^3 s^-1 at 1e4 K */
} or_atom;

typedef struct {
  double t_exp;
  const double* T_e, *n_e;        /* [C] */
  const double* n_species;        /* [C*S] */
  const double* gamma_ion;        /* [C*S*3] */
  const double* gamma_pe;         /* [C*T] or NULL */
  const double* gamma_pi;         /* [C*N] or NULL: photoionisation of each level to
                                     the next stage's ground, s^-1, added to gamma_ion */
} or_cells;

/* ---- Photoionising levels (Sec. 2.3.1; Eq. A5) ------------------------------
 * For every species, stages 0 and 1 below its top stage (no ionisation from
 * the doubly ionised stage): the first max_per_stage levels of the stage, in
 * level order, that lie below the stage's ionisation energy ion_energy[s*3+z]
 * (erg). Writes (when not NULL) the global level, the threshold wavelength
 * h c / (E_ion - E_i) in cm and the hydrogenic cross section at threshold
 * 7.9e-18 (1 - E_i / E_ion)^-1/2 / (z + 1)^2 cm^2 of each; returns how many. */
int32_t oracle_pi_levels(const or_atom* a, const double* ion_energy, int32_t max_per_stage,
                         int32_t* level, double* lambda_thr, double* sigma0);

/* Solves cells [first, first+count). pops [C*N] in: initial guess (used when
 * use_guess != 0), out: solution. status[c]: 0 converged, 2 failed, 3 empty.
 * iters[c] (optional) receives the largest iteration count (fixed-point
 * plus Newton steps) over the cell's species. */
int oracle_nlte(const or_atom* a, const or_cells* cells, int64_t first, int64_t count,
                int use_guess, int max_iter, double tol, int nthreads,
                double* pops, int32_t* status, int32_t* iters);

/* Cold start (Boltzmann within each ion stage, stage ratios from a
 * ground-state-only balance). */
void oracle_nlte_cold(const or_atom* a, const or_cells* cells, int64_t c, double* pops_cell);

/* Rate matrix R[i*Ns+j] (i -> j, per atom in i, s^-1) of one species in one
 * cell at populations n (local numbering), exposed for the pins. */
void oracle_rate_matrix(const or_atom* a, const or_cells* cells, int64_t c, int32_t s,
                        const double* n_local, double* R);

/* GTH stationary vector of a generator given by off-diagonal rates R (row i -> j). */
void oracle_gth(int32_t N, const double* R, double* pi);

/* ---- Deterministic emission (Sec. 2.3; Eq. A3) ----------------------------
 * Line emission of each cell binned in wavelength: n_lambda bins, logarithmic
 * over [lambda_min, lambda_max); transition t (lambda_t in the range) emits
 * A_t beta_S(tau_t(n)) n_u V photons s^-1 of energy h c / lambda_t (Eq. A3 with
 * Delta E = h c / lambda_t) into bin floor(n_lambda ln(lambda_t / lambda_min) /
 * ln(lambda_max / lambda_min)). Outputs: bin_energy [C * n_lambda] erg s^-1;
 * bin_lambda [n_lambda], the reddest transition wavelength in each bin (0 if
 * none); outside [C], erg s^-1 of transitions outside the range. pops [C*N].
 * V is volumes[c] (cm^3, per cell) when volumes is not NULL, else cell_volume. */
void oracle_emission_bins(const or_atom* a, int64_t n_cells, const double* pops, double t_exp,
                          double cell_volume, const double* volumes, double lambda_min,
                          double lambda_max, int32_t n_lambda, double* bin_energy,
                          double* bin_lambda, double* outside);

/* Rays of the deterministic emission as explicit packets (x, y, z, n_x, n_y,
 * n_z, lambda_e, w0): for each cell c in [first, first + count), each bin b
 * with energy, each viewer k (theta-major: k = i_theta n_phi + i_phi) one ray
 * from the middle of the cell (origins[3 (c - first) ..] when origins is not
 * NULL, else the centre of the cube's cell) towards the viewer at theta =
 * (i_theta + 1/2) pi /
 * n_theta, phi = (i_phi + 1/2) 2 pi / n_phi, starting at the bin's reddest
 * wavelength with N = E_bin (Delta Omega_k / 4 pi) / (h c / lambda_b) photons
 * s^-1 (reading of the ray weight E_bin / Delta Omega_k / E_phot), Delta
 * Omega_k = (2 pi / n_phi)(cos theta_lo - cos theta_hi). Returns the number of
 * rays written to *packets (malloc'ed; free with oracle_free). */
int64_t oracle_ray_packets(int32_t n, double beta_max, const double* origins, int64_t first,
                           int64_t count, int32_t n_lambda, const double* bin_energy,
                           const double* bin_lambda, int32_t n_theta, int32_t n_phi,
                           double** packets);

/* ---- Batched NLTE problem (one element, three ion stages per cell) -------
 * Sec. 2.2 rate model with frozen rates: every bound-bound pair of a stage has
 * collisions (detailed balance upward), 20 % of pairs are radiative (A and a
 * photoexcitation rate, photo-de-excitation by detailed balance, beta = 1);
 * every level of stage z ionises to the ground of z+1; the ground of z+1
 * recombines into stage z, 1/3 to the ground and 2/3 over the excited levels
 * by statistical weight. Per-level and per-pair values are drawn from Philox
 * (key seed, 6) by the definition in batched.c. Levels are numbered cell by
 * cell, stage by stage, ground first. */
typedef struct {
  int64_t n_cells;
  uint64_t seed;
  const int32_t* level_count;     /* [C*3], stage 0 >= 1, absent stages last */
  const double* T_e;              /* [C] */
  const double* n_e;              /* [C] */
  const double* gamma_ion;        /* [C*2] */
  double alpha0[2];
  const double* gpe_table;        /* [n_gpe] photoexcitation rates a radiative pair draws from */
  int64_t n_gpe;
} or_batched;

/* Dense rate matrix R[i*N+j] (i -> j, s^-1) of cell c, N = levels of the cell. */
void oracle_batched_matrix(const or_batched* p, int64_t c, double* R);

/* Stationary populations (sum 1) of cells [first, first+count) by GTH on the
 * dense N x N matrix; pops indexed by the cell's first level pop_offset[c].
 * Returns the number of cells whose reduction hit a non-positive pivot. */
int64_t oracle_batched(const or_batched* p, const int64_t* pop_offset, int64_t first,
                       int64_t count, int nthreads, double* pops);

#endif
