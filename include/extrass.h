/* extrass.h - C ABI of the MI355X (gfx950) hot path of ExTraSS
 * (van Baal & Jerkstrand, arXiv 2511.07539): Monte Carlo photon-packet
 * transport through homologous 3D ejecta with Sobolev line absorption,
 * photoexcitation-rate estimators per (cell, line), and the per-cell NLTE
 * statistical-equilibrium solve that consumes them.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (HIP global memory on the handle's
 *    device) unless a comment says "host". They are owned by the caller; the
 *    library never frees them and keeps no pointer after the call's stream
 *    work has finished.
 *  - Scratch memory comes from the caller's workspace (`ws`, `ws_bytes`),
 *    sized by the matching *_workspace query. The library performs no device
 *    allocation during these calls.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream), so
 *    that this header needs no HIP header. All work is enqueued on it;
 *    outputs are valid once the stream has completed.
 *  - Return codes: EXTRASS_OK, or a negative EXTRASS_E* code (below). Bad
 *    arguments are detected on the host before any work is enqueued. Errors
 *    found on the device (e.g. a full record buffer) are reported through the
 *    `stats` output, documented per entry point. No C++ exception crosses
 *    this interface.
 *  - Units are CGS: wavelengths in cm, densities in cm^-3, rates in s^-1,
 *    time in s. The velocity coordinate is x = v/c; the grid is the cube
 *    [-beta_max, beta_max]^3 cut into n^3 equal cells, cell c = i + n*(j + n*k)
 *    with lower corner -beta_max + (i, j, k) * 2*beta_max/n.
 */
#ifndef EXTRASS_H
#define EXTRASS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXTRASS_OK 0
#define EXTRASS_EINVAL (-1)      /* invalid argument (null pointer, bad size, unsorted lines) */
#define EXTRASS_ENOSPACE (-2)    /* workspace smaller than the query returned */
#define EXTRASS_EHIP (-3)        /* a HIP runtime call failed; see extrass_last_error */
#define EXTRASS_EUNSUPPORTED (-4) /* size outside what the kernels support */

typedef struct extrass_ctx* extrass_handle;
typedef struct extrass_atom_ctx* extrass_atom_handle;

/* Creates a handle bound to HIP device `device` (reads its properties once).
 * *out receives the handle; destroy it with extrass_destroy. */
int extrass_create(extrass_handle* out, int device);
int extrass_destroy(extrass_handle h);
/* Static text for a return code. */
const char* extrass_error_string(int code);
/* Detail of the last error reported through `h` (host string owned by h). */
const char* extrass_last_error(extrass_handle h);

/* ------------------------------------------------------------------------
 * Transport (Sec. 2.3 "Radiative transfer", Sec. 2.3.2 "Photoexcitation").
 *
 * Packets travel in straight lines (no scattering) through homologous flow.
 * With first-order Doppler shifts, D = n.x grows by exactly the path length,
 * and line k (rest wavelength lambda_k) comes into resonance at
 * D_k = 1 - lambda_lab / lambda_k. Lines are visited in wavelength order,
 * starting at the first line redward of the emission wavelength; in cell c a
 * line is tested when D_k lies in (D, D_exit] of the packet's segment in that
 * cell. A line with tau(c,k) > 1e-4 absorbs dN = w (1 - e^-tau) of the
 * packet's w photons, leaving w e^-tau; est[c,k] receives dN / f_corr; the packet stops once
 * w * lambda_e < 1e-6 * w0 * lambda_k (remaining comoving energy below 1e-6 of
 * its start), and escapes when it leaves the cube.
 *
 * Opacity: tau(c,k) = line_tau0[k] * tau_scale[c] (f_corr = 1), except for
 * lines with line_trans[k] = t >= 0 when tau_ct is given: then
 * tau = tau_ct[c*n_trans + t], f_corr = fcorr_ct[c*n_trans + t] (Eq. A2 and
 * its stimulated-emission factor; see extrass_line_tau). An entry of
 * line_trans outside [-1, n_trans) is never used as an index: the line is
 * treated as a background line and stats[EXTRASS_STAT_BAD_LINES] is set
 * (the estimators are then invalid).
 */
typedef struct {
  int32_t n;                    /* cells per axis (1..1024) */
  double beta_max;              /* cube half-width, in units of c */
  const float* tau_scale;       /* [C] */
  const double* cell_photons;   /* [C] photons s^-1 emitted by the cell */
  const int32_t* cell_packets;  /* [C] packets emitted by the cell, >= 0 */
  int32_t n_lines;              /* L >= 0 */
  const double* line_lambda;    /* [L] rest wavelengths, cm, non-decreasing */
  const float* line_tau0;       /* [L] */
  const int32_t* line_trans;    /* [L] transition of each line or -1; may be NULL */
  int32_t n_trans;              /* T (only with tau_ct) */
  const double* tau_ct;         /* [C*T] or NULL */
  const double* fcorr_ct;       /* [C*T] or NULL (then f_corr = 1) */
  const struct extrass_photoion* photoion;  /* host struct: photoionisation opacity of the
                                               cells (below), or NULL for none */
  const struct extrass_spherical* spherical; /* host struct: a spherical grid instead of the
                                                cube (below; n and beta_max are then not
                                                read), or NULL */
} extrass_grid;

/* Spherical grid (Sec. 2: the paper's (r, theta, phi) cells, larger at large
 * radii). Shells between r_edge[i] and r_edge[i+1] (x = v/c, r_edge[0] = 0),
 * polar bins between theta_edge[j] and theta_edge[j+1] (0 = theta_0 < ... <
 * theta_{n_theta} = pi), n_phi equal azimuthal slices [2 pi k / n_phi,
 * 2 pi (k+1) / n_phi). Cell c = i_r + n_r (i_theta + n_theta i_phi), so a phi
 * slice is a contiguous range of cells; C = n_r n_theta n_phi for every [C]
 * array of the grid. A packet leaves its cell where its straight path first
 * meets a bounding sphere, cone or half-plane while moving out of the cell,
 * steps to the neighbour across it (phi wraps around), and escapes beyond the
 * outer sphere. Sampled emission in a cell takes r^3 uniform between the
 * shell's edges (u0), cos(theta) uniform in the polar bin (u1) and phi
 * uniform in the slice (u2) for the position; the direction, wavelength and
 * weight are drawn as in the cube. Explicit packets start in the cell their
 * position falls in; one beyond the outer sphere is dropped and flagged
 * (EXTRASS_STAT_BAD_PACKETS). Deterministic rays start at the middle of the
 * cell: mid-radius, mid-angle of the polar bin, mid-slice. Spherical grids run
 * with FP64 positions and distances (geometry_fp32 is ignored).
 * extrass_transport_streamed splits them into n_domains equal ranges of
 * phi (Sec. 2.4.1's phi decomposition; each a contiguous range of cells). */
typedef struct extrass_spherical {
  int32_t n_r, n_theta, n_phi;  /* each >= 1; C at most 2^31 - 1 */
  const double* r_edge;         /* device [n_r + 1], increasing */
  const double* theta_edge;     /* device [n_theta + 1], increasing */
  int32_t n_domains;            /* streamed transport: phi subdomains, >= 2, dividing n_phi
                                   (not read elsewhere) */
} extrass_spherical;

/* Photoionisation in the transport (Sec. 2.3.1; Eq. A5). M photoionising
 * levels, numbered in order of non-decreasing threshold wavelength lambda_j;
 * level j has the hydrogenic cross section sigma_j(lambda) = sigma0_j
 * (lambda / lambda_j)^3 blueward of its threshold and zero redward. Every
 * move of a packet -- to a wall, or to a line that interacts (tau > 1e-4) --
 * passes through the continuum: level j absorbs while the comoving wavelength
 * is below lambda_j (the move is cut where the packet redshifts past it),
 * tau_j = a_j integral(lambda^3 ds) times `length`, a_j = n_j sigma0_j /
 * lambda_j^3 with n_j the level's population density in the cell. The move
 * absorbs w (1 - e^-tau), tau = sum_j tau_j, shared in proportion to tau_j,
 * and leaves w e^-tau. After a move that ends at a wall the packet stops when
 * its comoving energy is below 1e-6 of its start (w lambda_e < 1e-6 w0
 * lambda_comoving), as after a line. Photons absorbed by photoionisation are
 * counted in stats[EXTRASS_STAT_W_PI].
 * opacity (extrass_pi_opacity writes it): per cell, 2M + 1 doubles: the
 * suffix sums S_j = sum_{k >= j} a_k for j = 0..M (S_M = 0), then a_0..a_{M-1}
 * (cm^-4). tally: per cell 2M doubles accumulated into: T_0..T_{M-1}, then
 * Q_0..Q_{M-1}, such that level j absorbed a_j (sum_{k <= j} T_k + Q_j)
 * photons s^-1 in the cell (extrass_pi_rates turns them into rates). */
typedef struct extrass_photoion {
  int32_t n_levels;             /* M, 1..4096 */
  const double* lambda_thr;     /* device [M] threshold wavelengths, cm, non-decreasing */
  const double* opacity;        /* device [C*(2M+1)] */
  double length;                /* cm per unit of path (x = v/c): c t_exp */
  double* tally;                /* device [C*2M], accumulated into */
} extrass_photoion;

/* Emission. Sampled mode (explicit_packets == NULL): packet ids are cell-major,
 * cell c owning ids [sum_{c'<c} cell_packets[c'], ... + cell_packets[c]).
 * Packet p (j-th of its cell's n_c) draws two Philox4x64-10 blocks with key
 * (seed, 3) and counters (p, iteration, 0, 0), (p, iteration, 1, 0); with
 * u_i = (r_i >> 11) * 2^-53: position corner + h*(u0, u1, u2), direction
 * mu = 2*u3 - 1, phi = 2*pi*u4, wavelength
 * lambda_lo + (lambda_hi - lambda_lo) * (j + u5) / n_c, weight
 * cell_photons[c] / n_c. Explicit mode: packet p is the row
 * explicit_packets[8p .. 8p+7] = (x, y, z, nx, ny, nz, lambda_e, w0).
 * Runs packets [first_packet, first_packet + n_packets). */
typedef struct extrass_rays extrass_rays;  /* deterministic rays, below */
typedef struct {
  uint64_t seed;
  int32_t iteration;
  int64_t first_packet;
  int64_t n_packets;
  double lambda_lo, lambda_hi;      /* emission band, cm */
  const double* explicit_packets;   /* [P*8] or NULL */
  int32_t geometry_fp32;            /* 0: FP64 positions and distances; 1: FP32 */
  const extrass_rays* rays;         /* host struct: deterministic rays instead of sampled
                                       packets (explicit_packets NULL), or NULL */
} extrass_source;

/* Deterministic emission (Sec. 2.3): every cell sends one ray per wavelength
 * bin with emission and per viewer, from the middle of the cell, starting at
 * the reddest wavelength of the bin's lines (no absorption in its own line)
 * and carrying the bin's photons times the viewer's share of the sphere.
 * Viewers: n_theta x n_phi, theta_a = (a + 1/2) pi / n_theta, phi_b =
 * (b + 1/2) 2 pi / n_phi, solid angle dOmega = (2 pi / n_phi)(cos(a pi /
 * n_theta) - cos((a + 1) pi / n_theta)). Ray r (packet id) of cell
 * c = r / (B V), bin slot j = (r / V) mod B, viewer k = r mod V (theta-major,
 * k = a n_phi + b), V = n_theta n_phi, carries
 * bin_photons[c*B + j] * dOmega_k / (4 pi) photons s^-1 (the reading of the
 * weight E_bin / dOmega_k / E_phot as E_bin (dOmega_k / 4 pi) / E_phot, so a
 * bin's rays carry its photons once over the sphere); rays of zero weight are
 * skipped (no events, not tallied). Valid ray ids are [0, C B V). */
struct extrass_rays {
  int32_t n_theta, n_phi;       /* viewers, 1..4096 each */
  int32_t n_bins;               /* B, occupied wavelength bins */
  const double* bin_lambda;     /* device [B] starting (comoving) wavelength of each bin, cm */
  const double* bin_photons;    /* device [C*B] photons s^-1 each cell emits in each bin */
};

/* Transport statistics, written to `stats` (device, EXTRASS_STATS doubles). */
enum {
  EXTRASS_STAT_W_EMIT = 0,   /* photons s^-1 emitted */
  EXTRASS_STAT_W_ESC = 1,    /* escaped */
  EXTRASS_STAT_W_KILL = 2,   /* left in packets stopped by the 1e-6 rule */
  EXTRASS_STAT_W_ABS = 3,    /* absorbed in lines (sum of dN) */
  EXTRASS_STAT_N_INTER = 4,  /* line interactions (tau > 1e-4 resonances) */
  EXTRASS_STAT_N_CHECKS = 5, /* line resonances tested */
  EXTRASS_STAT_N_CROSS = 6,  /* cell-to-cell crossings */
  EXTRASS_STAT_N_ESCAPED = 7,
  EXTRASS_STAT_N_KILLED = 8,
  EXTRASS_STAT_E_ESC = 9,    /* escaped weight over lab wavelength, sum of w / lambda_L
                                (cm^-1 s^-1): h c times it is the escaping luminosity */
  EXTRASS_STAT_W_PI = 10,    /* absorbed by photoionisation (grid.photoion) */
  EXTRASS_STAT_QUEUE_FULL = 13,  /* streamed transport: 1.0 if an octant queue overflowed */
  EXTRASS_STAT_BAD_PACKETS = 14, /* 1.0 if some packet id lay beyond the sampling plan
                                    or a packet had no wall ahead (NaN or zero direction);
                                    such packets are dropped */
  EXTRASS_STAT_BAD_LINES = 15,   /* 1.0 if line_lambda is not non-decreasing, or a line_trans
                                    entry lies outside [-1, n_trans) (est invalid) */
  EXTRASS_STATS = 16
};

/* Bytes of workspace extrass_transport needs for this problem. */
size_t extrass_transport_workspace(const extrass_grid* g, const extrass_source* s);

/* Runs the packets and OVERWRITES est[C*L] (cell-major, FP64) with their
 * photoexcitation counts (photons s^-1 absorbed per cell and line, divided by
 * f_corr). stats[EXTRASS_STATS] is overwritten. packets_out, if not NULL,
 * receives EXTRASS_PACKET_FIELDS doubles per packet, packet first_packet + i
 * at record i: escaped weight (0 if stopped), lab wavelength (cm), weight at
 * the stop (0 if escaped), absorbed photons, the lab-frame direction n_x, n_y,
 * n_z (unchanged along the ray; FP32-rounded with geometry_fp32), and 0.
 * Packets dropped as bad leave their record untouched. Host structs `g` and
 * `s` are read during the call only. */
enum { EXTRASS_PACKET_FIELDS = 8 };
int extrass_transport(extrass_handle h, const extrass_grid* g, const extrass_source* s,
                      double* est, double* stats, double* packets_out, void* ws,
                      size_t ws_bytes, void* stream);

/* extrass_transport without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments, outputs and errors as
 * extrass_transport; the scratch is a 16 MiB array the library keeps on each
 * GPU for the life of the process (set up by extrass_create), and
 * EXTRASS_ENOSPACE is returned when extrass_transport_workspace(g, s) exceeds
 * it (a 100^3 grid with 30000 lines and 1e8 packets needs 10.1 MiB; 120^3
 * fits, 125^3 does not). Allocates nothing. Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other handles, other threads) race and must be serialised by the caller. */
int extrass_transport_noalloc(extrass_handle h, const extrass_grid* g, const extrass_source* s,
                              double* est, double* stats, double* packets_out, void* stream);

/* ------------------------------------------------------------------------
 * Emergent spectra per viewer (Sec. 2.3: rays leave towards 20 x 20 viewers
 * spread evenly in polar and azimuthal angle; the emission is binned
 * logarithmically in wavelength; global convergence compares the total
 * energy in the emergent spectra with the deposition). Each escaped packet
 * record (escaped weight w > 0) of `packets` (device, the layout
 * extrass_transport writes) is assigned to the viewer bin of its direction,
 * theta = acos(n_z) in n_theta equal bins of [0, pi] and
 * phi = atan2(n_y, n_x) mod 2 pi in n_phi equal bins of [0, 2 pi), and to
 * the wavelength bin floor(n_lambda ln(lambda_L / lambda_min) /
 * ln(lambda_max / lambda_min)) when lambda_min <= lambda_L < lambda_max
 * (others are not binned). photons (if not NULL) receives w, energy (if not
 * NULL) w h c / lambda_L (erg s^-1), both ADDED at
 * [(i_theta * n_phi + i_phi) * n_lambda + i_lambda] (device,
 * n_theta * n_phi * n_lambda doubles; zero them first). Dividing by a
 * viewer's solid angle, 2 pi / n_phi (cos theta_lo - cos theta_hi), and by
 * 4 pi gives the isotropic-equivalent rates. Bins: 1..4096 per angle,
 * 1..2^20 in wavelength, 0 < lambda_min < lambda_max; EXTRASS_EINVAL
 * otherwise.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_theta, n_phi, n_lambda;
  double lambda_min, lambda_max;   /* cm */
} extrass_spectrum_bins;

int extrass_spectrum(extrass_handle h, const double* packets, int64_t n_packets,
                     const extrass_spectrum_bins* bins, double* photons, double* energy,
                     void* stream);

/* ------------------------------------------------------------------------
 * Line emission for the deterministic rays (Sec. 2.3; Eq. A3): the
 * bound-bound emissivity A_ul Delta E_ul beta_S N_u of every atom transition,
 * N_u = n_u V the cell's atoms in the upper level, beta_S from Eqs. A1-A2 at
 * the cell's populations, Delta E_ul = h c / lambda_ul, binned by wavelength
 * in n_lambda logarithmic bins over [lambda_min, lambda_max) (bin
 * floor(n_lambda ln(lambda / lambda_min) / ln(lambda_max / lambda_min))).
 * A plan fixes the binning for an atom: its occupied bins (those holding at
 * least one transition), in increasing order, each starting its rays at the
 * reddest transition wavelength in it. */
typedef struct extrass_emission_ctx* extrass_emission_plan;
int extrass_emission_plan_create(extrass_handle h, extrass_atom_handle atom, double lambda_min,
                                 double lambda_max, int32_t n_lambda, extrass_emission_plan* out);
int extrass_emission_plan_destroy(extrass_emission_plan p);
/* B, and (host arrays of capacity B, either may be NULL) each occupied bin's
 * number in the n_lambda grid and its starting wavelength; *device_lambda
 * (may be NULL) receives the plan's device copy of the wavelengths [B], for
 * extrass_rays.bin_lambda (owned by the plan). */
int extrass_emission_plan_info(extrass_emission_plan p, int32_t* n_bins, int32_t* bin_number,
                               double* bin_lambda, const double** device_lambda);
/* For the grid's cells (the cube: C = n^3, V = (2 beta_max / n c t_exp)^3;
 * a spherical grid: each cell's own volume (c t_exp)^3 (r_b^3 - r_a^3) / 3
 * (cos theta_a - cos theta_b) 2 pi / n_phi) at
 * populations pops [C*N]: bin_photons [C*B] (device, overwritten) photons
 * s^-1 per occupied bin, E_bin / (h c / lambda_bin); outside [C] (device, may
 * be NULL) erg s^-1 emitted in lines outside [lambda_min, lambda_max). */
int extrass_emission(extrass_handle h, extrass_emission_plan p, extrass_atom_handle atom,
                     const extrass_grid* grid, double t_exp, const double* pops,
                     double* bin_photons, double* outside, void* stream);

/* ------------------------------------------------------------------------
 * Photoionising levels and their opacity (Sec. 2.3.1; Eq. A5). Ionisation is
 * taken from stages 0 and 1 of each species (none from the doubly ionised
 * stage upwards), from the first max_per_stage levels of each such stage (in
 * level order) that lie below the stage's ionisation energy ion_energy[s*3+z]
 * (erg, host [S*3]; from the stage's ground to the next stage's ground). Each
 * takes the hydrogenic cross section of Eq. A5 (Verner and TOPBASE data are
 * not used): at threshold lambda_j = h c / (E_ion - E_j),
 * sigma0_j = 7.9e-18 (1 - E_j / E_ion)^-1/2 / (z + 1)^2 cm^2. A plan holds
 * them in order of non-decreasing threshold (equal thresholds in level order).
 * EXTRASS_EINVAL if no level qualifies or max_per_stage < 1. */
typedef struct extrass_pi_ctx* extrass_pi_plan;
int extrass_pi_plan_create(extrass_handle h, extrass_atom_handle atom, const double* ion_energy,
                           int32_t max_per_stage, extrass_pi_plan* out);
int extrass_pi_plan_destroy(extrass_pi_plan p);
/* M, and (host arrays of capacity M, each may be NULL) each level's global
 * index, threshold wavelength (cm) and sigma0 (cm^2), in the plan's order;
 * *device_lambda (may be NULL): the plan's device copy of the thresholds,
 * for extrass_photoion.lambda_thr (owned by the plan). */
int extrass_pi_plan_info(extrass_pi_plan p, int32_t* n_levels, int32_t* level, double* lambda_thr,
                         double* sigma0, const double** device_lambda);
/* The opacity table of extrass_photoion for n_cells cells at populations
 * pops [C*N] (cm^-3): opacity [C*(2M+1)] (device, overwritten). */
int extrass_pi_opacity(extrass_handle h, extrass_pi_plan p, int64_t n_cells, const double* pops,
                       double* opacity, void* stream);
/* Photoionisation rates per atom of each level from a transport's tally:
 * gamma_pi[c*N + i] = N_abs / (n_i V) = sigma0_j / lambda_j^3 (sum_{k <= j}
 * T_k + Q_j) / V for the plan's level j = i, 0 for levels outside the plan
 * (the population cancels). V as in extrass_rates, from grid (n, beta_max)
 * and t_exp. tally [C*2M], gamma_pi [C*N] (device, overwritten). For
 * extrass_cells.gamma_pi. */
int extrass_pi_rates(extrass_handle h, extrass_pi_plan p, const extrass_grid* grid, double t_exp,
                     const double* tally, double* gamma_pi, void* stream);

/* ------------------------------------------------------------------------
 * Eq. A2: tau_S = (A_ul / 8 pi) (g_u / g_l) lambda^3 n_l (1 - g_l n_u / (g_u n_l)) t
 * for every (cell, transition), with f_corr = 1 - g_l n_u / (g_u n_l) (the
 * stimulated-emission correction of the photoexcitation count). pops is
 * [C*N] (number densities per level); a cell with n_l <= 0 gets tau = 0,
 * f_corr = 1. Outputs tau_ct, fcorr_ct [C*T]. Atoms of more than 8192 levels
 * return EXTRASS_EUNSUPPORTED (a cell's populations are staged in LDS). */
int extrass_line_tau(extrass_handle h, extrass_atom_handle atom, int64_t n_cells,
                     const double* pops, double t_exp, double* tau_ct, double* fcorr_ct,
                     void* stream);

/* ------------------------------------------------------------------------
 * Rates (Sec. 2.3.1-2.3.2): photons absorbed per second in a cell's line,
 * divided by the number of atoms in the line's lower level (population times
 * cell volume), is the photoexcitation rate per lower atom:
 *   gamma_pe[c*T + t] = est[c*L + line(t)] / (pops[c*N + lower(t)] * V),
 * 0 where that population is 0. The cells are those of `grid` (C = n^3,
 * L = grid->n_lines; only n, beta_max and n_lines are read), and V is the
 * physical volume of one cell in homologous flow, (2 beta_max / n * c t_exp)^3
 * cm^3 (a cell's width in x = v/c times c t_exp), computed here. est [C*L],
 * pops [C*N], gamma_pe [C*T] are device arrays. EXTRASS_EINVAL if an atom
 * transition's line index is not below L. The photo-de-excitation rate per
 * upper atom follows by detailed balance, (g_l/g_u) gamma_pe, inside the NLTE
 * solve. */
int extrass_rates(extrass_handle h, extrass_atom_handle atom, const extrass_grid* grid,
                  double t_exp, const double* est, const double* pops, double* gamma_pe,
                  void* stream);

/* ------------------------------------------------------------------------
 * Streamed transport over velocity octants (Sec. 2.4 decomposes the grid
 * into subdomains; here the subdomains are the 8 octants of the cube, visited
 * one after another on one GPU so that only one octant's estimator table
 * is resident).
 *
 * Runs the packets of the whole sampling plan (first_packet 0, n_packets =
 * sum of cell_packets; explicit packets are not supported) through the cube,
 * one octant at a time: an octant's visit emits its own cells' packets (first
 * visit), resumes the packets queued for it, accumulates into est_octant and
 * queues every packet that crosses into another octant. Rounds of visits,
 * forwards and backwards in octant order in turn, repeat until no packet is
 * queued (at most 4 rounds: a straight ray crosses each coordinate plane
 * once). Packets keep their ids, Philox streams
 * and arithmetic, so the events equal those of extrass_transport.
 *
 * After each visit, if atom is not NULL, the visit's estimators are turned
 * into photoexcitation rates and ADDED to gamma_pe[C*T] (zeroed at the start;
 * rates are linear in the estimators): gamma_pe[c,t] += est/(n_l V), with V
 * the cell volume (2 beta_max / n * c t_exp)^3 as in extrass_rates. If
 * est_global is not NULL ([C*L], tests and small grids), every visit's table
 * is also added into it at the global cell rows (zeroed at the start).
 *
 * n: even. est_octant: device [(n/2)^3 * L] (local cell i + (n/2)(j + (n/2) k)
 * within the octant, octant o = (i >= n/2) + 2 (j >= n/2) + 4 (k >= n/2)).
 * A spherical grid is split instead into its n_domains equal phi ranges (the
 * paper's phi decomposition), visited in rounds as the octants, for at most
 * n_domains + 1 rounds (each range is convex); est_octant is then
 * [C / n_domains * L], the subdomain's cells in their global order, and V is
 * each cell's own volume.
 * est_octant may be NULL when only the rates are wanted (atom given,
 * est_global NULL, the grid's tau_ct/line_trans set and line_trans the
 * inverse of the atom's transition -> line map, else EXTRASS_EINVAL): each
 * interaction on an atom line then adds dN / f_corr straight into
 * gamma_pe[c,t], which is divided by n_l V at the end. No octant table is
 * kept and no flush runs; lines of no atom transition are not recorded. The
 * rates equal the table path's up to the order of the additions and the
 * division, taken as a product with 1 / (n_l V) (atoms of more than 8192
 * levels: EXTRASS_EUNSUPPORTED).
 * queue_capacity: packets each subdomain's queue holds; the workspace holds one
 * queue of 120-byte records per subdomain. A full queue loses packets: stats[QUEUE_FULL]
 * is set and the call returns EXTRASS_ENOSPACE. The host waits for the stream
 * once per round of visits (the queue lengths decide whether another round
 * runs). */
size_t extrass_transport_streamed_workspace(const extrass_grid* grid, int64_t queue_capacity);
int extrass_transport_streamed(extrass_handle h, const extrass_grid* grid, const extrass_source* src,
                               extrass_atom_handle atom, const double* pops, double t_exp,
                               double* est_octant, double* est_global, double* gamma_pe,
                               double* stats, int64_t queue_capacity, void* ws, size_t ws_bytes,
                               void* stream);

/* ------------------------------------------------------------------------
 * Atom (Sec. 2.2: all ion stages of a species are solved together). HOST
 * arrays; extrass_atom_create copies them to the device once. Levels of all
 * species are numbered globally; species s owns [species_offset[s],
 * species_offset[s+1]), at most 64 levels per species, ion stages 0..2 in
 * order, each stage's first level its ground state. Each transition joins two
 * levels of one stage (lower < upper), at most one transition per pair. */
typedef struct {
  int32_t n_species;
  const int32_t* species_offset;   /* host [S+1] */
  int32_t n_levels;
  const int32_t* level_ion;        /* host [N] */
  const double* level_energy;      /* host [N] erg above the stage's ground */
  const double* level_g;           /* host [N] */
  int32_t n_trans;
  const int32_t* trans_lower;      /* host [T] */
  const int32_t* trans_upper;      /* host [T] */
  const double* trans_A;           /* host [T] s^-1 */
  const double* trans_lambda;      /* host [T] cm */
  const double* trans_upsilon;     /* host [T] effective collision strength */
  const int32_t* trans_line;       /* host [T] line index (>= 0; below the grid's L where
                                      extrass_rates or the streamed rates use it) */
  const double* ion_alpha0;        /* host [S*3] recombination into stage z at 1e4 K */
} extrass_atom_desc;

int extrass_atom_create(extrass_handle h, const extrass_atom_desc* desc, extrass_atom_handle* out);
int extrass_atom_destroy(extrass_atom_handle a);

/* Cell state for the NLTE solve (device arrays). */
typedef struct {
  int64_t n_cells;
  double t_exp;                 /* s */
  const double* T_e;            /* [C] K */
  const double* n_e;            /* [C] cm^-3 */
  const double* n_species;      /* [C*S] cm^-3 */
  const double* gamma_ion;      /* [C*S*3] s^-1, stage z -> z+1 from any level */
  const double* gamma_pe;       /* [C*T] s^-1 per lower atom, or NULL */
  const double* gamma_pi;       /* [C*N] s^-1 per atom: photoionisation of each level to the
                                   next stage's ground (extrass_pi_rates), added to
                                   gamma_ion for that level; or NULL */
} extrass_cells;

typedef struct {
  int32_t max_iter;    /* iteration cap per species (fixed-point + Newton) */
  double tol;          /* convergence: the last Newton correction max |d ln n| and the
                          fixed-point residual max |P(n)/n - 1| both below tol; the
                          populations are then within about tol relative of the root */
  int32_t use_guess;   /* 1: start from pops on entry (a non-positive entry means
                          the cold start for that system); 0: cold start */
  int32_t factor_fp32; /* 0: every reduction in FP64. 1: the mixed-precision pass:
                          the fixed-point steps, except the first from a guess,
                          reduce their stationary problem in FP32 (positive numbers
                          only, so each population keeps FP32's relative accuracy;
                          the matrix is scaled by one power of two to a largest
                          entry in [1, 2), the reference ground's population is
                          2^100). Residuals and Newton systems stay FP64, so the
                          exit test, and the accuracy tol, are those of 0. A step
                          with an FP32 pivot or population outside the normal
                          range is assembled again and reduced in FP64. Stage-block
                          atoms only (blocks of at most 32 states in 64 lanes),
                          else EXTRASS_EUNSUPPORTED */
  int32_t warm_budget; /* with use_guess: after this many iterations from the guess,
                          a system still in its fixed-point phase or with a
                          fixed-point residual above 1e-6 restarts from the cold
                          start with the iterations left (status 1); so does one
                          whose line search stalls before. 0: never, and the guess
                          is taken as near the root (a previous solution): the
                          fixed-point steps continue until they change no
                          population by more than 0.1 in log n (1.0 with a
                          budget) before Newton starts */
} extrass_nlte_opts;

/* Statistical equilibrium per cell and species (Sec. 2.2, Eqs. A1-A2):
 * the positive root of inflow = outflow for every level with
 * sum_i n_i = n_species, rates
 *   R_ul += A_ul beta_S(tau_ul(n)) + n_e q_ul + (g_l/g_u) Gamma_PE,
 *   R_lu += n_e q_lu + Gamma_PE,  q_ul = 8.629e-6 Upsilon / (g_u sqrt(T)),
 *   q_lu = q_ul (g_u/g_l) exp(-(E_u - E_l)/kT),
 *   ionisation stage z -> ground of z+1 at gamma_ion (plus gamma_pi of the
 *   level when given), recombination from the
 *   ground of z+1 at n_e alpha0 (T/1e4)^-0.8, 1/3 to the ground state of z and
 *   2/3 over its excited levels by statistical weight (Appendix A.2).
 * pops [C*N]: in = guess (if use_guess), out = solution. status [C]: 0
 * converged, 1 converged after falling back to the cold start, 2 not
 * converged within max_iter, 3 empty cell (all species 0).
 * iters [C] (may be NULL): largest iteration count over the cell's species. */
size_t extrass_nlte_workspace(extrass_atom_handle a, int64_t n_cells);
int extrass_nlte_solve(extrass_handle h, extrass_atom_handle a, const extrass_cells* cells,
                       const extrass_nlte_opts* opts, double* pops, int32_t* status,
                       int32_t* iters, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method): an MLP
 * 6 -> 256 -> 256 -> 256 -> 100 with SiLU hidden layers maps normalised cell
 * features to normalised log10(n_i / n_species) of a 100-level, 2-species
 * atom. Parameters: one FP32 vector of extrass_mlp_param_count() values,
 * W1 [256*6], b1 [256], W2 [256*256], b2, W3 [256*256], b3, W4 [100*256],
 * b4 [100], weights row-major [out][in]. GEMMs run on BF16 matrix cores with
 * FP32 accumulation; master weights and optimiser state are FP32. */
size_t extrass_mlp_param_count(void);
size_t extrass_mlp_workspace(int64_t batch);
/* y [batch*100] = MLP(x [batch*6]) (x already normalised). */
int extrass_mlp_forward(extrass_handle h, const float* params, const float* x, float* y,
                        int64_t batch, void* ws, size_t ws_bytes, void* stream);
/* One training step on a batch with loss = mean((MLP(x) - t)^2) over all outputs:
 * adds the batch loss to *loss (device float; may be NULL), writes the
 * gradient to grad [P] when not NULL, and, when adam_m/adam_v [P] are given,
 * applies Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with `step`
 * >= 1) with learning rate lr to params. */
int extrass_mlp_train_step(extrass_handle h, float* params, float* adam_m, float* adam_v,
                           int32_t step, float lr, const float* x, const float* t, int64_t batch,
                           float* loss, float* grad, void* ws, size_t ws_bytes, void* stream);
/* Warm-start populations for extrass_nlte_solve (use_guess = 1): features of
 * each cell (log10 of the total species density, T_e, n_e and the deposition
 * [C] in erg s^-1 cm^-3, and the two species' number fractions), normalised by
 * norm[0..5] (means) and norm[6..11] (standard deviations), pass through the
 * MLP; outputs are de-normalised with norm[12..111] (means) and
 * norm[112..211] (standard deviations), exponentiated and scaled so that each
 * species sums to its density. The atom must have 2 species and 100 levels. */
size_t extrass_nlte_warm_start_workspace(int64_t n_cells);
/* The six raw (not normalised) features extrass_nlte_warm_start forms for each
 * cell, x [n_cells*6] (device, FP32), for building training sets and their
 * normalisation. The atom must have 2 species. */
int extrass_mlp_features(extrass_handle h, extrass_atom_handle atom, const extrass_cells* cells,
                         const double* deposition, float* x, void* stream);
int extrass_nlte_warm_start(extrass_handle h, extrass_atom_handle atom, const extrass_cells* cells,
                            const double* deposition, const float* params, const float* norm,
                            double* pops, void* ws, size_t ws_bytes, void* stream);

/* ---- Batched NLTE solve: one element with three ion stages per cell -------
 * The ion stages of an element are solved together (Sec. 2.2) under frozen
 * rates: the linear problem that each fixed-point or Newton step of the
 * statistical-equilibrium iteration solves. Cells have different level
 * counts; all cells are solved by one persistent batched factorisation.
 *
 * Rate model (per atom, s^-1), with per-level and per-pair values drawn from
 * Philox4x64-10 under key (seed, 6), uniforms u_k = (x_k >> 11) 2^-53:
 *   level i of stage z in cell c, counter (c, z, i, 2^63):
 *     g = 1 + floor(9 u0); E = 0 (ground, i = 0) or 69 k T_e u1
 *   pair l < u of stage z, counter (c, z, l, u): radiative iff u0 < 0.2, with
 *     A = 10^(-3 + 11 u1), Gamma_PE = gamma_pe_table[min(n - 1, floor(u3 n))]
 *     (n = n_gamma_pe); q = 10^(-10 + 3 u2)
 *   upper (higher E; higher index on a tie) -> lower: A + n_e q + (g_l/g_u) Gamma_PE
 *   lower -> upper: n_e q (g_u/g_l) exp(-(E_u - E_l)/kT) + Gamma_PE
 *   every level of stage z -> ground of z+1: gamma_ion[c*2 + z]
 *   ground of z+1 -> level i of z: n_e alpha0[z] (T_e/1e4)^-0.8 x
 *     (1/3 for the ground; (2/3) g_i / sum of g over the excited levels)
 * Output: stationary populations, summing to 1 per cell, cell after cell,
 * stage after stage, ground first: level i of stage z of cell c at
 * sum_{c'<c} (L0+L1+L2)(c') + sum_{z'<z} L_z'(c) + i.
 *
 * Method: stages are coupled only through the next stage's ground state, so
 * the excited levels of each stage are eliminated in a block of their own
 * (state reduction with pivots formed as sums of off-diagonal rates,
 * Grassmann-Taksar-Heyman; blocked, trailing updates on matrix cores), the
 * ground states form a birth-death chain, and back-substitution recovers the
 * rest. In exact arithmetic this is the reduction of the full N x N matrix in
 * an order that skips its structural zeros. */
typedef struct {
  int64_t n_cells;
  uint64_t seed;                 /* Philox key word 0 */
  const int32_t* level_count;    /* HOST [C*3] levels of stages 0..2; stage 0 >= 1;
                                    absent stages (0) only after present ones; <= 1023 */
  const int32_t* level_count_d;  /* device copy of level_count */
  const double* T_e;             /* device [C] K */
  const double* n_e;             /* device [C] cm^-3 */
  const double* gamma_ion;       /* device [C*2] s^-1 */
  double alpha0[2];              /* cm^3 s^-1 at 1e4 K, recombination into stage z */
  const double* gamma_pe_table;  /* device [n_gamma_pe] s^-1, ascending: the photoexcitation
                                    rates a radiative pair takes its rate from (rates
                                    measured from the estimators of a transport run) */
  int64_t n_gamma_pe;            /* >= 1, else EXTRASS_EINVAL */
} extrass_batched;

typedef struct {
  int32_t factor_fp32;  /* 0: FP64 factorisation; 1: FP32 factorisation (FP32 matrix
                           cores) with FP64 residuals and iterative refinement */
  int32_t refine;       /* refinement sweeps with factor_fp32 (each: residual, correction) */
  double tol;           /* status 1 when the last correction exceeds tol relative, componentwise */
  int32_t panel;        /* panel width 16, 32 or 64; 0 = tuned value (extrass_batched_tune) or 32 */
  int32_t per_cu;       /* resident work-groups per compute unit; 0 = tuned value or 2 */
} extrass_batched_opts;

/* Workspace: *min_bytes solves one cell at a time; *all_bytes holds every
 * cell at once. Any size in between works; cells are then solved in chunks. */
int extrass_batched_workspace(extrass_handle h, const extrass_batched* p,
                              const extrass_batched_opts* o, size_t* min_bytes, size_t* all_bytes);

/* pops: device [sum of all level counts] out. status: device [C] out: 0 solved, 1 solved but
 * the last refinement correction exceeded tol, 2 failed (non-positive pivot or
 * non-finite result). EINVAL for bad counts or pointers, ENOSPACE for a
 * workspace below *min_bytes. Stream-ordered; the host waits only for the
 * upload of the chunk plan. */
int extrass_batched_solve(extrass_handle h, const extrass_batched* p, const extrass_batched_opts* o,
                          double* pops, int32_t* status, void* ws, size_t ws_bytes,
                          void* stream);

/* Autotuner: times the factorisation of the first cells of p (up to the
 * workspace's capacity) for every panel width (16, 32, 64) and work-groups per
 * compute unit (1, 2, 4) in the precision o->factor_fp32, keeps the fastest in
 * the handle (used when panel/per_cu are 0) and reports it in choice[0..1];
 * times[9] (optional, host) receives the milliseconds of each candidate, panel-major.
 * Synchronises the stream. */
int extrass_batched_tune(extrass_handle h, const extrass_batched* p, const extrass_batched_opts* o,
                         void* ws, size_t ws_bytes, void* stream, int32_t* choice,
                         float* times);

#ifdef __cplusplus
}
#endif
#endif
