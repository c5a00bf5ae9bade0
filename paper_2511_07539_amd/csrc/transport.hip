// Monte Carlo packet transport with Sobolev line absorption (Sec. 2.3; the
// photoexcitation estimators of Sec. 2.3.2, the continuum of Sec. 2.3.1).
//
// One persistent kernel: every lane follows one packet at a time, one event
// per loop trip (either the next line resonance inside the current cell or
// the crossing of the cell wall). When a lane's packet stops, the wave hands
// it the next packet id from a wave-private pool of ids, refilled from a
// global counter 256 ids at a time; a ballot over the wave finds the idle
// lanes and a popcount gives each its slot, so lanes refill without one
// atomic per packet and the wave stays full until the ids run out.
//
// Geometry (positions, directions, distances, Doppler coordinate D) runs in
// the template type G: double for the reference path, float for the fast
// path. Weights, estimators and the line wavelength arithmetic stay FP64.
//
// Octant mode (velocity-space subdomains streamed through HBM): the kernel
// follows only packets inside one subdomain, an octant of the cube or a
// range of phi slices of the spherical grid, and accumulates into that
// subdomain's estimator table (or straight into the rates). A packet that
// crosses into another subdomain is stored, whole, in that subdomain's queue
// and continues when it is visited. Subdomains are convex, so a straight ray
// never returns to one it has left (a cube's ray visits at most four
// octants). Emitted packets keep their global ids and Philox streams, and a
// stored packet resumes with the same arithmetic, so the split run takes
// the same events as the unsplit one.
//
// The spherical grid (Sec. 2) replaces the wall search by the first exit
// root among the cell's spheres, cones and half-planes (sph_exit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include <mutex>

#include "atom.hpp"
#include "common.hpp"
#include "philox.hpp"

namespace extrass {
namespace {

constexpr double kTauMin = 1e-4;    // lines with tau > 1e-4 interact
constexpr double kKillFrac = 1e-6;  // stop below 1e-6 of the starting energy
constexpr int kPool = 256;          // ids taken from the global counter per refill
constexpr int kRefill = 32;         // idle lanes that trigger a refill
// Wavelength lookup bins for the first line above lambda_e: a power of two at
// least 4 per line, between 1024 and 2^18 (at most 1 MB of table).
static inline int lam_bins(int L) {
  int n = 1024;
  while (n < 4 * L && n < (1 << 18)) n <<= 1;
  return n;
}
constexpr int kBlock = 256;
constexpr int kPkFields = 8;         // doubles per packet record

struct alignas(16) LineRec {
  double inv_lam;
  int32_t trans;
  float tau0;
};

struct TArgs {
  int n;
  double beta, h;
  const float* tau_scale;
  const double* cell_photons;
  const int32_t* cell_packets;
  int L;
  const double* lam;
  const LineRec* lines;  // [L] per line: 1/lambda, transition (-1: tau0 x tau_scale), tau0
  int T;
  const double* tau_ct;
  const double* fcorr_ct;
  uint64_t seed;
  uint32_t iteration;
  int64_t first, count;  // packet ids [first, first + count) (a streamed visit reads its
                          // count from `visit`)
  double lam_lo, lam_hi;
  const double* explicit_pk;
  // deterministic rays (ray_ph not NULL): B occupied bins, viewers nt x np
  const double* ray_lam;   // [B]
  const double* ray_ph;    // [C*B]
  int ray_B, ray_nt, ray_np;
  const int64_t* start;  // [C+1] exclusive prefix of cell_packets
  const int32_t* lam_bin;   // [nbin] first line above each log-lambda bin edge (lowered)
  const double* lam_par;    // lambda_0, bins per unit lambda
  int nbin;
  const int32_t* chunk_cell;  // [nchunk] cell of packet first + 256 j (sampled mode)
  int64_t nchunk;
  int64_t C;
  double* est;
  double* stats;
  double* pk_out;
  unsigned long long* queue;
  // streamed visits (oct >= 0: the subdomain visited)
  int oct, half;
  int lo[3];                 // first cell index of the octant per axis
  int sub_slices;            // spherical grid: phi slices per subdomain (0: octants of the cube)
  int64_t sub_c0;            // spherical grid: first cell of the current subdomain
  int64_t n_emit;            // packets emitted in this visit (first visit only)
  const int64_t* ostart;     // [Coct+1] prefix of cell_packets over the octant's cells
  const int64_t* visit;      // [2] set on the device before the visit: packets in
                             // the visit (emitted + resumed), first queued record
  struct QPk* qbase;         // one queue of qcap records per subdomain
  unsigned long long* qtail; // [subdomains] queue tails
  int64_t qcap;
  uint8_t* touched;          // [Coct] rows that received an estimator this visit
  double* gdirect;           // octant mode without a table: [C*T] sums of dN / f_corr per
                             // (cell, atom transition); other lines are not recorded
  // photoionisation (the PI kernels): M thresholds, per-cell opacity rows and
  // tally rows (the layout of extrass_photoion), cm per unit of path
  int pi_M;
  const double* pi_lam;
  const double* pi_opac;
  double* pi_tally;
  double pi_len;
  // spherical grid (the SPH kernels): shell and polar edges, slice width
  int sph_nr, sph_nt, sph_np;
  const double* sph_r;   // [nr + 1]
  const double* sph_th;  // [nt + 1]
  const double* sph_cth; // [nt + 1] cos of the polar edges (workspace)
  const double* sph_cs;  // [2 (np + 1)] cos, sin of the azimuthal edges (workspace)
  double sph_dphi;
};

// A packet in flight between subdomains: the whole state after a wall crossing.
struct QPk {
  double x[3], d[3], D, lamL, lam_e, w, w0, wabs;
  int32_t ci[3], k;
  int64_t pid;
};
static_assert(sizeof(QPk) == 120, "queue record layout");

// ---- small helper kernels -------------------------------------------------

// The line list packed into one 16-byte record per line, so that the event
// loop's line test and opacity choice take one load.
// A line_trans entry outside [-1, n_trans) is never used as an index: the line
// becomes a background line (k_check_lines flags the estimators invalid).
__global__ void k_prep(const double* lam, const float* tau0, const int32_t* line_trans,
                       int has_ct, int n_trans, LineRec* lines, int L, double* stats,
                       unsigned long long* queue) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < EXTRASS_STATS) stats[t] = 0.0;
  if (t == 0) *queue = 0ull;
  for (int k = t; k < L; k += gridDim.x * blockDim.x) {
    LineRec r;
    r.inv_lam = 1.0 / lam[k];
    const int tr = has_ct ? line_trans[k] : -1;
    r.trans = (tr < -1 || tr >= n_trans) ? -1 : tr;
    r.tau0 = tau0[k];
    lines[k] = r;
  }
}

// Runs after k_prep (which clears stats): flags a line list that is not
// non-decreasing, or a line -> transition entry outside [-1, n_trans).
__global__ void k_check_lines(const double* lam, const int32_t* line_trans, int has_ct,
                              int n_trans, int L, double* stats) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = t; k < L; k += gridDim.x * blockDim.x) {
    const bool unsorted = k > 0 && !(lam[k] >= lam[k - 1]);
    const int tr = has_ct ? line_trans[k] : -1;
    if (unsorted || tr < -1 || tr >= n_trans) stats[EXTRASS_STAT_BAD_LINES] = 1.0;
  }
}

// Lookup for the first line above a wavelength: bin b of [lambda_0,
// lambda_{L-1}] (uniform bins) stores the first line above its lower edge,
// lowered by 1e-9 relative. The search starts one bin below the wavelength's
// own, so rounding in the bin index or the edge can only start the forward
// scan early, never late.
__global__ void k_lambin(const double* lam, int L, int nbin, int32_t* bin, double* par) {
  const double l0 = L > 0 ? lam[0] : 0.0;
  const double span = L > 1 ? lam[L - 1] - l0 : 0.0;
  const double inv = span > 0.0 ? nbin / span : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    par[0] = l0;
    par[1] = inv;
  }
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nbin; b += gridDim.x * blockDim.x) {
    const double edge = inv > 0.0 ? (l0 + b / inv) * (1.0 - 1e-9) : 0.0;
    int lo = 0, hi = L;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (lam[mid] > edge) hi = mid;
      else lo = mid + 1;
    }
    bin[b] = lo;
  }
}

// Sampled mode: cell of packet first + 256 j, so that a packet's cell search
// starts from the cells of its 256-id chunk.
__global__ void k_chunk_cells(const int64_t* start, int64_t C, int64_t first, int64_t nchunk,
                              int32_t* chunk_cell) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nchunk;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = first + (j << 8);
    int64_t lo = 0, hi = C;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (start[mid] <= p) lo = mid;
      else hi = mid;
    }
    chunk_cell[j] = (int32_t)lo;
  }
}

// Exclusive prefix of cell_packets in three launches: sums of tiles of
// kScanTile cells, an exclusive scan of the tile sums (one workgroup), then
// each tile's scan plus its offset. Cells are taken in the grid's order, or
// with oct >= 0 over octant oct's cells in local order (i + half (j + half k)).
constexpr int kScanTile = 1024;  // 256 threads x 4 cells

__device__ __forceinline__ int64_t scan_count(const int32_t* counts, int64_t r, int n, int oct) {
  if (oct < 0) return counts[r];
  const int half = n / 2;
  const int i = (int)(r % half), j = (int)((r / half) % half), k = (int)(r / ((int64_t)half * half));
  const int o0 = (oct & 1) ? half : 0, o1 = (oct & 2) ? half : 0, o2 = (oct & 4) ? half : 0;
  return counts[(i + o0) + (int64_t)n * ((j + o1) + (int64_t)n * (k + o2))];
}

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Exclusive scan of the 256 values of a workgroup of 256 threads; the total
// goes to *total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* wsum, int64_t* total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t inc = wave_incl_scan(v, lane);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int64_t off = 0;
  for (int w = 0; w < wave; ++w) off += wsum[w];
  if (total) *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  return off + inc - v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t* counts, int64_t C, int n,
                                                   int oct, int64_t* tsum) {
  __shared__ int64_t wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  int64_t v = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (base + j < C) v += scan_count(counts, base + j, n, oct);
  int64_t tot = 0;
  block_excl_scan(v, wsum, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// One workgroup of 256: exclusive scan of nt tile sums in place, total to *end.
__global__ __launch_bounds__(256) void k_scan_sums(int64_t* tsum, int64_t nt, int64_t* end) {
  __shared__ int64_t wsum[4];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nt; b0 += 256) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nt ? tsum[i] : 0;
    int64_t tot = 0;
    const int64_t ex = block_excl_scan(v, wsum, &tot);
    if (i < nt) tsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *end = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* counts, int64_t C, int n,
                                                   int oct, const int64_t* tsum, int64_t* start) {
  __shared__ int64_t wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  int64_t c[4], v = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    c[j] = base + j < C ? scan_count(counts, base + j, n, oct) : 0;
    v += c[j];
  }
  int64_t run = tsum[blockIdx.x] + block_excl_scan(v, wsum, nullptr);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < C) start[base + j] = run;
    run += c[j];
  }
}

// start[0..m) = exclusive prefix of the m counts, start[m] = their total.
void scan_counts(hipStream_t st, const int32_t* counts, int64_t m, int n, int oct, int64_t* tsum,
                 int64_t* start) {
  const int64_t nt = (m + kScanTile - 1) / kScanTile;
  if (nt > 0)
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(256), 0, st, counts, m, n, oct, tsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, st, tsum, nt, start + m);
  if (nt > 0)
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(256), 0, st, counts, m, n, oct, tsum,
                       start);
}


// After an octant visit, for every row the visit touched: add its rates into
// gamma (atom lines) and, if asked, the row into the global table; then zero
// the row, so that the octant table is all zero again for the next visit.
// One work-group per row; untouched rows return at once.
__global__ __launch_bounds__(256) void k_octant_flush(double* __restrict__ eo, uint8_t* touched,
                                                      int n, int oct, int64_t c0, int L, int N,
                                                      int T, const int32_t* __restrict__ lo,
                                                      const int32_t* __restrict__ line,
                                                      const double* __restrict__ pops,
                                                      CellVolume V, double* __restrict__ gamma,
                                                      double* __restrict__ eg) {
  const int64_t r = blockIdx.x;
  if (!touched[r]) return;
  int64_t c = c0 + r;  // a phi subdomain (c0 >= 0): contiguous cells
  if (c0 < 0) {        // an octant of the cube
    const int half = n / 2;
    const int o0 = (oct & 1) ? half : 0, o1 = (oct & 2) ? half : 0, o2 = (oct & 4) ? half : 0;
    const int i = (int)(r % half), j = (int)((r / half) % half), k = (int)(r / ((int64_t)half * half));
    c = (i + o0) + (int64_t)n * ((j + o1) + (int64_t)n * (k + o2));
  }
  double* row = eo + r * L;
  const double Vc = gamma ? V(c) : 0.0;
  if (gamma)
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
      const double Nl = pops[c * N + lo[t]] * Vc;
      if (Nl > 0.0) gamma[c * T + t] += row[line[t]] / Nl;
    }
  if (eg)
    for (int q = threadIdx.x; q < L; q += blockDim.x) eg[c * L + q] += row[q];
  __syncthreads();
  for (int q = threadIdx.x; q < L; q += blockDim.x) row[q] = 0.0;
  if (threadIdx.x == 0) touched[r] = 0;
}

// Rates from the direct sums: gamma_pe[c,t] = sum(dN / f_corr) / (n_l V).
// One work-group per cell row: the reciprocals 1 / (n_l V) of the cell's
// levels go to LDS once, then the row is scaled in place (coalesced). Empty
// levels give zero rates.
__global__ __launch_bounds__(256) void k_rates_direct(int64_t C, int N, int T,
                                                     const int32_t* __restrict__ lo,
                                                     const double* __restrict__ pops,
                                                     CellVolume V, double* __restrict__ gamma) {
  extern __shared__ double inv[];  // [N]
  for (int64_t c = blockIdx.x; c < C; c += gridDim.x) {
    const double vc = V(c);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const double Nl = pops[c * N + i] * vc;
      inv[i] = Nl > 0.0 ? 1.0 / Nl : 0.0;
    }
    __syncthreads();
    double* g = gamma + c * T;
    for (int t = threadIdx.x; t < T; t += blockDim.x) g[t] = g[t] * inv[lo[t]];
    __syncthreads();
  }
}

// The direct sums need the grid's line -> transition map to be the inverse of
// the atom's transition -> line map; flag[0] is set when it is not.
__global__ void k_check_map(const int32_t* __restrict__ line_trans, int L,
                            const int32_t* __restrict__ o_line, int T, unsigned long long* flag) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
    const int k = o_line[t];
    if (k < 0 || k >= L || line_trans[k] != t) flag[0] = 1ull;
  }
}

// Cosines of a spherical grid's polar edges, and cosines and sines of its
// azimuthal edges 2 pi k / np, k = 0..np.
__global__ void k_sph_trig(const double* th, int nt, int np, double* cth, double* cs) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= nt) cth[t] = cos(th[t]);
  if (t <= np) {
    double sp, cp;
    sincos(2.0 * M_PI * t / np, &sp, &cp);
    cs[2 * t] = cp;
    cs[2 * t + 1] = sp;
  }
}

__global__ void k_reset_u64(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

// Before a streamed visit of subdomain o: the visit's packets (ne emitted,
// plus those queued for o since its last visit, up to the queue's capacity)
// and the first of the queued records; the packet pool restarts.
__global__ void k_visit_begin(int o, int64_t ne, int64_t qcap, unsigned long long* counters,
                              int64_t* visit) {
  if (threadIdx.x != 0) return;
  const int64_t t = (int64_t)counters[1 + o];
  const int64_t avail = t < qcap ? t : qcap;
  int64_t* head = visit + 2;
  visit[0] = ne + (avail - head[o]);
  visit[1] = head[o];
  head[o] = avail;
  counters[0] = 0ull;
}

__global__ void k_zero(double* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)(blockIdx.x * blockDim.x + threadIdx.x);
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t n2 = n / 2;
  double2* p2 = reinterpret_cast<double2*>(p);
  for (int64_t j = i; j < n2; j += stride) p2[j] = make_double2(0.0, 0.0);
  if (i == 0 && (n & 1)) p[n - 1] = 0.0;
}

// ---- the transport kernel -------------------------------------------------

template <class G>
struct Packet {
  int ci[3];
  G x[3], d[3];
  G D, Dexit, s, smin, dist[3];
  double lamL, lam_e, w, w0, wabs;
  int k;
  bool have_exit;
  bool bad;
  // photoionisation (PI kernels only): D where the continuum absorption last
  // stopped, the first threshold redward of the comoving wavelength there,
  // and the photons absorbed
  double Dp, wpi;
  int jpi;
  int sbits;  // spherical grid: the boundaries the current segment ends on
};

// The record of line k, or an empty one past the red end of the list.
__device__ __forceinline__ LineRec line_rec(const TArgs& A, int k) {
  LineRec r;
  r.inv_lam = 0.0;
  r.trans = -1;
  r.tau0 = 0.0f;
  if (k < A.L) r = A.lines[k];
  return r;
}

// Per-packet record at the stop: escaped weight, lab wavelength, weight at a
// kill, photons absorbed in lines, the direction (lab frame; unchanged along
// the ray), and the photons absorbed by photoionisation (0 without it).
template <class G, bool PI = false>
__device__ __forceinline__ void put_record(double* o, const Packet<G>& q, double w_esc, double w_kill) {
  o[0] = w_esc;
  o[1] = q.lamL;
  o[2] = w_kill;
  o[3] = q.wabs;
  o[4] = (double)q.d[0];
  o[5] = (double)q.d[1];
  o[6] = (double)q.d[2];
  o[7] = PI ? q.wpi : 0.0;
}

template <class G>
__device__ __forceinline__ G wall(const TArgs& A, int i) {
  return static_cast<G>(-A.beta + static_cast<double>(i) * A.h);
}

// First line with lambda_k > lam: a table lookup one bin below lam's bin,
// then a forward scan (about one line per bin).
__device__ __forceinline__ int first_line_above(const TArgs& A, double lam) {
  const double x = (lam - A.lam_par[0]) * A.lam_par[1];
  int b = x > 0.0 ? (x < (double)A.nbin ? (int)x : A.nbin - 1) : 0;
  b = b > 0 ? b - 1 : 0;
  int k = A.lam_bin[b];
  while (k < A.L && A.lam[k] <= lam) ++k;
  return k;
}

// ---- spherical grid ---------------------------------------------------------

// Cell of point x on the spherical grid: the shell and polar bin whose lower
// edges lie at or below r and theta, and the slice holding phi; false beyond
// the outer sphere.
__device__ __forceinline__ bool sph_locate(const TArgs& A, const double x[3], int ci[3]) {
  const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  if (!(r < A.sph_r[A.sph_nr])) return false;
  int lo = 0, hi = A.sph_nr;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (A.sph_r[mid] <= r) lo = mid; else hi = mid;
  }
  ci[0] = lo;
  const double th = r > 0.0 ? acos(fmin(1.0, fmax(-1.0, x[2] / r))) : 0.0;
  lo = 0;
  hi = A.sph_nt;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (A.sph_th[mid] <= th) lo = mid; else hi = mid;
  }
  ci[1] = lo;
  double ph = atan2(x[1], x[0]);
  if (ph < 0.0) ph += 2.0 * M_PI;
  int k = static_cast<int>(floor(ph / A.sph_dphi));
  ci[2] = k < 0 ? 0 : (k > A.sph_np - 1 ? A.sph_np - 1 : k);
  return true;
}

// Path length s >= 0 from x along n to where the ray leaves spherical cell
// ci: the first root of one of its bounding surfaces at which the ray moves
// out of the cell (roots where it moves in, such as the surface it just
// crossed, do not count); `which` receives the surfaces met there (1 inner
// sphere, 2 outer sphere, 4 lower cone, 8 upper cone, 16 lower half-plane,
// 32 upper half-plane). A root within eps behind x counts as at x (x sits on
// that surface up to rounding).
__device__ __forceinline__ double sph_exit(const TArgs& A, const double x[3], const double n[3], const int ci[3],
                           int& which) {
  const double xx = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  const double b = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
  const double eps = 1e-14 * A.sph_r[A.sph_nr];
  double best = INFINITY;
  which = 0;
  auto take = [&](double s, int bit) {
    if (!(s >= -eps)) return;
    s = s > 0.0 ? s : 0.0;
    if (s < best) {
      best = s;
      which = bit;
    } else if (s == best) {
      which |= bit;
    }
  };
  {  // outer sphere: the larger root of |x + s n| = r
    const double r = A.sph_r[ci[0] + 1];
    const double disc = b * b - (xx - r * r);
    take(-b + sqrt(disc > 0.0 ? disc : 0.0), 2);
  }
  if (ci[0] > 0) {  // inner sphere: the smaller root
    const double r = A.sph_r[ci[0]];
    const double disc = b * b - (xx - r * r);
    if (disc >= 0.0) take(-b - sqrt(disc), 1);
  }
  // cones: the lower edge theta_lo bounds z <= cos(theta_lo) |x|, the upper
  // edge z >= cos(theta_hi) |x|; roots of (z + s n_z)^2 = c^2 |x + s n|^2 on
  // the cone's own nappe (z of the sign of c), or of z = 0 for theta = pi/2
  for (int side = 0; side < 2; ++side) {
    const int j = ci[1] + side;
    if (j == 0 || j == A.sph_nt) continue;
    const double c = A.sph_cth[j];
    const double sgn = side == 0 ? 1.0 : -1.0;  // g = sgn (c |x| - z) >= 0 inside
    if (fabs(c) < 1e-12) {
      // the equatorial plane: g = -sgn z, decreasing when sgn n_z > 0
      if (sgn * n[2] > 0.0) take(-x[2] / n[2], 4 << side);
      continue;
    }
    const double Aq = n[2] * n[2] - c * c;
    const double Bq = x[2] * n[2] - c * c * b;
    const double Cq = x[2] * x[2] - c * c * xx;
    double rt[2];
    int nr = 0;
    if (fabs(Aq) < 1e-300) {
      if (Bq != 0.0) rt[nr++] = -Cq / (2.0 * Bq);
    } else {
      const double disc = Bq * Bq - Aq * Cq;
      if (disc >= 0.0) {
        const double q = sqrt(disc);
        rt[nr++] = (-Bq - q) / Aq;
        rt[nr++] = (-Bq + q) / Aq;
      }
    }
    for (int i = 0; i < nr; ++i) {
      const double sr = rt[i];
      const double p[3] = {x[0] + sr * n[0], x[1] + sr * n[1], x[2] + sr * n[2]};
      if ((p[2] > 0.0) != (c > 0.0)) continue;  // the other nappe
      const double pr = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      if (!(pr > 0.0)) continue;
      const double dg = sgn * (c * (p[0] * n[0] + p[1] * n[1] + p[2] * n[2]) / pr - n[2]);
      if (dg < 0.0) take(sr, 4 << side);
    }
  }
  if (A.sph_np > 1) {  // half-planes through the z axis
    for (int side = 0; side < 2; ++side) {
      const double cp = A.sph_cs[2 * (ci[2] + side)], sp = A.sph_cs[2 * (ci[2] + side) + 1];
      // inside: counter-clockwise of the lower edge, clockwise of the upper
      const double sgn = side == 0 ? 1.0 : -1.0;
      const double g0 = sgn * (-sp * x[0] + cp * x[1]);
      const double g1 = sgn * (-sp * n[0] + cp * n[1]);
      if (!(g1 < 0.0)) continue;
      const double sr = -g0 / g1;
      const double px = x[0] + sr * n[0], py = x[1] + sr * n[1];
      if (cp * px + sp * py > 0.0) take(sr, 16 << side);
    }
  }
  return best;
}

// RAYS: the deterministic-ray kernel, compiled apart so that the sampled
// kernels keep their register allocation. SPH: the spherical grid.
template <class G, bool RAYS, bool SPH>
__device__ void emit(const TArgs& A, int64_t p, Packet<G>& q) {
  double x[3], d[3], lam_e, w0;
  int ci[3];
  q.bad = false;
  if (A.explicit_pk) {
    const double* e = A.explicit_pk + 8 * p;
    for (int a = 0; a < 3; ++a) {
      x[a] = e[a];
      d[a] = e[3 + a];
      int i = static_cast<int>(floor((e[a] + A.beta) / A.h));
      ci[a] = i < 0 ? 0 : (i > A.n - 1 ? A.n - 1 : i);
    }
    if (SPH && !sph_locate(A, x, ci)) {  // starts beyond the outer sphere
      q.bad = true;
      return;
    }
    lam_e = e[6];
    w0 = e[7];
  } else if (RAYS) {
    // ray r = (c B + j) V + k from the middle of cell c towards viewer k,
    // starting at bin j's wavelength with the viewer's share of its photons
    const int64_t V = (int64_t)A.ray_nt * A.ray_np;
    if (p >= A.C * A.ray_B * V) {
      q.bad = true;
      return;
    }
    const int64_t cb = p / V;
    const int k = static_cast<int>(p - cb * V);
    const int64_t c = cb / A.ray_B;
    const int j = static_cast<int>(cb - c * A.ray_B);
    if constexpr (SPH) {
      // the middle of the spherical cell: mid-radius, mid-angle, mid-slice
      ci[0] = static_cast<int>(c % A.sph_nr);
      ci[1] = static_cast<int>((c / A.sph_nr) % A.sph_nt);
      ci[2] = static_cast<int>(c / ((int64_t)A.sph_nr * A.sph_nt));
      const double rm = 0.5 * (A.sph_r[ci[0]] + A.sph_r[ci[0] + 1]);
      const double tm = 0.5 * (A.sph_th[ci[1]] + A.sph_th[ci[1] + 1]);
      const double pm = (ci[2] + 0.5) * A.sph_dphi;
      double stm, ctm, spm, cpm;
      sincos(tm, &stm, &ctm);
      sincos(pm, &spm, &cpm);
      x[0] = rm * stm * cpm;
      x[1] = rm * stm * spm;
      x[2] = rm * ctm;
    } else {
      ci[0] = static_cast<int>(c % A.n);
      ci[1] = static_cast<int>((c / A.n) % A.n);
      ci[2] = static_cast<int>(c / ((int64_t)A.n * A.n));
      for (int a = 0; a < 3; ++a) x[a] = -A.beta + (static_cast<double>(ci[a]) + 0.5) * A.h;
    }
    const int it = k / A.ray_np, ip = k - it * A.ray_np;
    const double th = (it + 0.5) * M_PI / A.ray_nt;
    const double ph = (ip + 0.5) * 2.0 * M_PI / A.ray_np;
    const double dom = (2.0 * M_PI / A.ray_np) *
                       (cos(it * M_PI / A.ray_nt) - cos((it + 1) * M_PI / A.ray_nt));
    double st, ct, sp, cp;
    sincos(th, &st, &ct);
    sincos(ph, &sp, &cp);
    d[0] = st * cp;
    d[1] = st * sp;
    d[2] = ct;
    lam_e = A.ray_lam[j];
    w0 = A.ray_ph[cb] * dom / (4.0 * M_PI);
  } else {
    if (p >= A.start[A.C]) {  // id beyond the sampling plan
      q.bad = true;
      return;
    }
    int64_t lo = 0, hi = A.C;
    if (A.chunk_cell) {  // the cells of the packet's 256-id chunk bound the search
      const int64_t jc = (p - A.first) >> 8;
      if (jc >= 0 && jc < A.nchunk) {
        lo = A.chunk_cell[jc];
        hi = jc + 1 < A.nchunk ? (int64_t)A.chunk_cell[jc + 1] + 1 : A.C;
      }
    }
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (A.start[mid] <= p) lo = mid;
      else hi = mid;
    }
    const int64_t c = lo;
    const int64_t j = p - A.start[c];
    const int nc = A.cell_packets[c];
    if (nc <= 0) {  // id beyond the sampling plan
      q.bad = true;
      return;
    }
    const u64x4 r0 = philox4x64_10((uint64_t)p, A.iteration, 0, 0, A.seed, 3);
    const u64x4 r1 = philox4x64_10((uint64_t)p, A.iteration, 1, 0, A.seed, 3);
    if constexpr (SPH) {
      // uniform in the cell's volume: r^3 over the shell, cos(theta) over the
      // polar bin, phi over the slice
      ci[0] = static_cast<int>(c % A.sph_nr);
      ci[1] = static_cast<int>((c / A.sph_nr) % A.sph_nt);
      ci[2] = static_cast<int>(c / ((int64_t)A.sph_nr * A.sph_nt));
      const double ra = A.sph_r[ci[0]], rb = A.sph_r[ci[0] + 1];
      const double r = cbrt(ra * ra * ra + unit53(r0.v[0]) * (rb * rb * rb - ra * ra * ra));
      const double ca = A.sph_cth[ci[1]], cb = A.sph_cth[ci[1] + 1];
      const double mu_x = ca + unit53(r0.v[1]) * (cb - ca);
      const double ph_x = 2.0 * M_PI * (ci[2] + unit53(r0.v[2])) / A.sph_np;
      const double sx = sqrt(fmax(0.0, 1.0 - mu_x * mu_x));
      double spx, cpx;
      sincos(ph_x, &spx, &cpx);
      x[0] = r * sx * cpx;
      x[1] = r * sx * spx;
      x[2] = r * mu_x;
    } else {
      ci[0] = static_cast<int>(c % A.n);
      ci[1] = static_cast<int>((c / A.n) % A.n);
      ci[2] = static_cast<int>(c / ((int64_t)A.n * A.n));
      for (int a = 0; a < 3; ++a)
        x[a] = (-A.beta + static_cast<double>(ci[a]) * A.h) + A.h * unit53(r0.v[a]);
    }
    const double mu = 2.0 * unit53(r0.v[3]) - 1.0;
    const double phi = 2.0 * M_PI * unit53(r1.v[0]);
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double sp, cp;
    sincos(phi, &sp, &cp);
    d[0] = st * cp;
    d[1] = st * sp;
    d[2] = mu;
    lam_e = A.lam_lo + (A.lam_hi - A.lam_lo) * ((static_cast<double>(j) + unit53(r1.v[1])) / nc);
    w0 = A.cell_photons[c] / nc;
  }
  for (int a = 0; a < 3; ++a) {
    q.ci[a] = ci[a];
    q.x[a] = static_cast<G>(x[a]);
    q.d[a] = static_cast<G>(d[a]);
  }
  const double D0 = d[0] * x[0] + d[1] * x[1] + d[2] * x[2];
  q.D = static_cast<G>(D0);
  q.lamL = lam_e * (1.0 - D0);
  q.lam_e = lam_e;
  q.w = w0;
  q.w0 = w0;
  q.wabs = 0.0;
  q.k = first_line_above(A, lam_e);
  q.have_exit = false;
}

struct Tally {
  double w_emit = 0, w_esc = 0, w_kill = 0, w_abs = 0, w_pi = 0;
  double e_esc = 0;  // escaped weight over lab wavelength: h c e_esc is the escaping erg s^-1
  uint32_t inter = 0, checks = 0, cross = 0, escaped = 0, killed = 0;  // per lane
  bool bad = false;
  bool overflow = false;
};

// Octant mode: the idx-th packet emitted in the octant (its cells in local
// order, each cell's packets in id order) is global packet start[c] + j.
__device__ __forceinline__ int64_t octant_packet(const TArgs& A, int64_t idx) {
  // a phi subdomain's cells are contiguous, and so are their packet ids
  if (A.sub_slices) return A.start[A.sub_c0] + idx;
  const int64_t Co = (int64_t)A.half * A.half * A.half;
  int64_t lo = 0, hi = Co;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (A.ostart[mid] <= idx) lo = mid;
    else hi = mid;
  }
  const int il = (int)(lo % A.half), jl = (int)((lo / A.half) % A.half), kl = (int)(lo / ((int64_t)A.half * A.half));
  const int64_t c = (il + A.lo[0]) + (int64_t)A.n * ((jl + A.lo[1]) + (int64_t)A.n * (kl + A.lo[2]));
  return A.start[c] + (idx - A.ostart[lo]);
}

template <class G>
__device__ void store(QPk* r, const Packet<G>& q, int64_t pid) {
  for (int a = 0; a < 3; ++a) {
    r->x[a] = (double)q.x[a];
    r->d[a] = (double)q.d[a];
    r->ci[a] = q.ci[a];
  }
  r->D = (double)q.D;
  r->lamL = q.lamL;
  r->lam_e = q.lam_e;
  r->w = q.w;
  r->w0 = q.w0;
  r->wabs = q.wabs;
  r->k = q.k;
  r->pid = pid;
}

// Values stored from G convert back exactly.
template <class G>
__device__ int64_t resume(const QPk& r, Packet<G>& q) {
  for (int a = 0; a < 3; ++a) {
    q.x[a] = static_cast<G>(r.x[a]);
    q.d[a] = static_cast<G>(r.d[a]);
    q.ci[a] = r.ci[a];
  }
  q.D = static_cast<G>(r.D);
  q.lamL = r.lamL;
  q.lam_e = r.lam_e;
  q.w = r.w;
  q.w0 = r.w0;
  q.wabs = r.wabs;
  q.k = r.k;
  q.have_exit = false;
  q.bad = false;
  return r.pid;
}

// First photoionisation threshold above the comoving wavelength lam.
__device__ __forceinline__ int pi_first_above(const TArgs& A, double lam) {
  int lo = 0, hi = A.pi_M;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (A.pi_lam[mid] > lam) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Integral of lambda^3 dD over a move D_a -> D_b of the ray, lambda(D) =
// lambda_L / (1 - D), lambda_a and lambda_b its ends: (1/2) lambda_a lambda_b
// (lambda_a + lambda_b) (D_b - D_a), the antiderivative lambda_L^3 / (2 (1 -
// D)^2) differenced without cancellation.
__device__ __forceinline__ double lam3_integral(double la, double lb, double dD) {
  return 0.5 * la * lb * (la + lb) * dD;
}

// Photoionisation over the move of the packet from q.Dp to Db in cell c (Sec.
// 2.3.1): the levels whose thresholds lie redward of the comoving wavelength
// absorb, those the packet redshifts past during the move only up to where it
// reaches them. Levels absorbing over the whole move share the suffix sum
// S_jb of the cell's opacity row; the cut ones (rare) are added one by one.
// Returns the move's optical depth (0: nothing absorbed).
template <class G>
__device__ __forceinline__ double pi_move(const TArgs& A, Packet<G>& q, int64_t c, double Db,
                                          Tally& t) {
  const double Da = q.Dp;
  q.Dp = Db;
  const int M = A.pi_M;
  if (!(Db > Da) || q.jpi >= M) return 0.0;
  const double lamL = q.lamL;
  const double la = lamL / (1.0 - Da);
  int j = q.jpi;
  while (j < M && A.pi_lam[j] <= la) ++j;
  const double lb = lamL / (1.0 - Db);
  int jb = j;
  while (jb < M && A.pi_lam[jb] < lb) ++jb;
  q.jpi = jb;
  if (j >= M) return 0.0;
  const double* row = A.pi_opac + c * (2 * M + 1);
  const double full = lam3_integral(la, lb, Db - Da) * A.pi_len;
  const double Sjb = jb < M ? row[jb] : 0.0;
  double tau = Sjb * full;
  for (int i = j; i < jb; ++i) {
    const double li = A.pi_lam[i];
    tau += row[M + 1 + i] * (lam3_integral(la, li, (1.0 - lamL / li) - Da) * A.pi_len);
  }
  if (!(tau > 0.0)) return 0.0;
  const double Nabs = q.w * (-expm1(-tau));
  const double r = Nabs / tau;
  double* tl = A.pi_tally + c * 2 * M;
  if (jb < M && Sjb > 0.0) atomicAdd(tl + jb, r * full);
  for (int i = j; i < jb; ++i) {
    const double li = A.pi_lam[i];
    if (row[M + 1 + i] > 0.0)
      atomicAdd(tl + M + i, r * (lam3_integral(la, li, (1.0 - lamL / li) - Da) * A.pi_len));
  }
  q.w = q.w * exp(-tau);
  q.wpi += Nabs;
  t.w_pi += Nabs;
  return tau;
}

// Three waves per SIMD: the kernel is bound by the latency of its gathers and
// scattered atomics, and the third wave (a few dwords of rarely used state
// spilled) is worth more than the spill.
template <class G, bool RAYS, bool PI, bool SPH, bool OCT>
__device__ __forceinline__ void transport_body(const TArgs& A) {
  const int lane = threadIdx.x & 63;
  Packet<G> q;
  LineRec nxt;  // record of line q.k, loaded ahead so that the event does not wait for it
  nxt.trans = -1;
  int64_t pid = -1;
  bool done = false;
  uint64_t pool_base = 0, pool_left = 0;
  bool exhausted = false;
  Tally t;
  const int64_t C = A.C;
  (void)C;
  // a streamed visit learns its size from the device (no host round trip)
  int64_t count = A.count;
  const QPk* inbox = nullptr;
  if constexpr (OCT) {
    count = A.visit[0];
    inbox = A.qbase + (int64_t)A.oct * A.qcap + A.visit[1];
    if (count == 0) return;
  }

  for (;;) {
    // ---- hand idle lanes new packet ids (ballot + popcount over the wave).
    // Emission is a chain of dependent loads (cell search, first line) plus
    // two Philox blocks; a packet lives only a few events, so refilling as
    // soon as one lane is idle would run emission for a few lanes almost
    // every event. Lanes wait until half the wave is idle (or no lane is
    // busy, or the ids are used up): 4.0 -> 3.5 ms for fill + transport of
    // 1e7 packets at 50^3, with the same tallies.
    const bool need = (pid < 0) && !done;
    uint64_t m = __ballot(need);
    if (m && (exhausted || __popcll(m) >= kRefill || m == __ballot(!done))) {
      if (pool_left == 0 && !exhausted) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(A.queue, (unsigned long long)kPool);
        base = __shfl(base, 0);
        pool_base = base;
        pool_left = base >= (uint64_t)count ? 0 : ((uint64_t)count - base < (uint64_t)kPool
                                                     ? (uint64_t)count - base : (uint64_t)kPool);
        if (pool_left == 0) exhausted = true;
      }
      const int rank = __popcll(m & ((1ull << lane) - 1ull));
      const uint64_t cnt = __popcll(m);
      const uint64_t take = cnt < pool_left ? cnt : pool_left;
      if (need) {
        if ((uint64_t)rank < take) {
          const int64_t idx = (int64_t)(pool_base + rank);
          if (OCT && idx >= A.n_emit) {
            pid = resume<G>(inbox[idx - A.n_emit], q);
            nxt = line_rec(A, q.k);
            if constexpr (PI) {  // absorbed up to the wall it came through
              q.Dp = (double)q.D;
              q.jpi = pi_first_above(A, q.lamL / (1.0 - q.Dp));
              q.wpi = 0.0;
            }
          } else {  // one emission site for both modes keeps the register peak down
            const int64_t p = !OCT ? A.first + idx : octant_packet(A, idx);
            emit<G, RAYS, SPH>(A, p, q);
            if (q.bad) {
              t.bad = true;
              pid = -1;
            } else if (RAYS && !(q.w0 > 0.0)) {  // a ray with no photons: skipped
              pid = -1;
            } else {
              pid = p;
              t.w_emit += q.w0;
              nxt = line_rec(A, q.k);
              if constexpr (PI) {
                q.Dp = (double)q.D;
                q.jpi = pi_first_above(A, q.lam_e);
                q.wpi = 0.0;
              }
            }
          }
        } else if (exhausted) {
          done = true;
        }
      }
      pool_base += take;
      pool_left -= take;
    }
    if (__ballot(!done) == 0ull) break;
    if (pid < 0) continue;

    // ---- events of this lane's packet. A lane whose segment has no line
    // left before the wall crosses it, and the line test of the new segment
    // follows in the same pass, so that a pass of the wave does a crossing
    // and a line event where the packet's next two events are those. The
    // order of events of each packet is unchanged.
    bool stop = false;
    bool line_event = q.have_exit && q.k < A.L && static_cast<G>(1.0 - q.lamL * nxt.inv_lam) <= q.Dexit;
    if constexpr (PI) {
      if (q.have_exit && !line_event) {
        // the continuum up to the wall, in the cell being left; then the
        // 1e-6 rule on the comoving energy left there
        const int64_t c = SPH ? q.ci[0] + (int64_t)A.sph_nr * (q.ci[1] + (int64_t)A.sph_nt * q.ci[2])
                              : q.ci[0] + (int64_t)A.n * (q.ci[1] + (int64_t)A.n * q.ci[2]);
        const double Db = (double)q.Dexit;
        if (pi_move<G>(A, q, c, Db, t) > 0.0 && q.w * q.lam_e * (1.0 - Db) < (kKillFrac * q.w0) * q.lamL) {
          t.w_kill += q.w;
          t.killed++;
          if (A.pk_out) put_record<G, PI>(A.pk_out + kPkFields * (pid - A.first), q, 0.0, q.w);
          stop = true;
        }
      }
    }
    if (q.have_exit && !line_event && !stop) {
      bool out = false;
      if constexpr (SPH) {
        // move to the exit point and across the surfaces met there
        for (int a = 0; a < 3; ++a) q.x[a] = q.x[a] + q.s * q.d[a];
        const int w = q.sbits;
        if (w & 1) q.ci[0] -= 1;
        if (w & 2) q.ci[0] += 1;
        if (w & 4) q.ci[1] -= 1;
        if (w & 8) q.ci[1] += 1;
        if (w & 16) q.ci[2] = q.ci[2] == 0 ? A.sph_np - 1 : q.ci[2] - 1;
        if (w & 32) q.ci[2] = q.ci[2] == A.sph_np - 1 ? 0 : q.ci[2] + 1;
        out = q.ci[0] >= A.sph_nr;
        if (q.ci[0] < 0 || q.ci[1] < 0 || q.ci[1] >= A.sph_nt) {  // rounding at the origin or a pole
          q.ci[0] = q.ci[0] < 0 ? 0 : q.ci[0];
          q.ci[1] = q.ci[1] < 0 ? 0 : (q.ci[1] >= A.sph_nt ? A.sph_nt - 1 : q.ci[1]);
        }
      } else {
      for (int a = 0; a < 3; ++a) {
        if (q.dist[a] == q.smin) {
          if (q.d[a] > G(0)) {
            q.ci[a] += 1;
            q.x[a] = wall<G>(A, q.ci[a]);
          } else {
            q.x[a] = wall<G>(A, q.ci[a]);
            q.ci[a] -= 1;
          }
          if (q.ci[a] < 0 || q.ci[a] >= A.n) out = true;
        } else {
          q.x[a] = q.x[a] + q.s * q.d[a];
        }
      }
      }
      q.D = q.Dexit;
      q.have_exit = false;
      if (out) {
        t.w_esc += q.w;
        t.e_esc += q.w / q.lamL;
        t.escaped++;
        if (A.pk_out) put_record<G, PI>(A.pk_out + kPkFields * (pid - A.first), q, q.w, 0.0);
        stop = true;
      } else {
        t.cross++;
        if constexpr (OCT) {
          const int dst = A.sub_slices ? q.ci[2] / A.sub_slices
                                       : (q.ci[0] >= A.half) | ((q.ci[1] >= A.half) << 1) |
                                             ((q.ci[2] >= A.half) << 2);
          if (dst != A.oct) {  // hand the packet to its next subdomain
            // one atomic per destination and wave: the lanes handing over to
            // the first lane's destination take consecutive slots, then the
            // rest repeat (a per-lane atomic on a handful of shared tails
            // serialised in L2: 152 -> 110 ms for a streamed 98 304-cell sphere)
            unsigned long long slot = 0;
            for (;;) {
              const int d0 = __builtin_amdgcn_readfirstlane(dst);
              const uint64_t same = __ballot(dst == d0);
              if (dst == d0) {
                const int leader = __ffsll((long long)same) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(A.qtail + d0, (unsigned long long)__popcll(same));
                base = __shfl(base, leader);
                slot = base + __popcll(same & ((1ull << lane) - 1ull));
                break;
              }
            }
            if ((int64_t)slot < A.qcap) store<G>(A.qbase + (int64_t)dst * A.qcap + (int64_t)slot, q, pid);
            else t.overflow = true;
            pid = -1;
            continue;
          }
        }
      }
    }
    if (!stop && !q.have_exit) {  // a new packet, or a new segment after a crossing
      G smin = static_cast<G>(INFINITY);
      if constexpr (SPH) {
        const double xd[3] = {(double)q.x[0], (double)q.x[1], (double)q.x[2]};
        const double nd[3] = {(double)q.d[0], (double)q.d[1], (double)q.d[2]};
        smin = static_cast<G>(sph_exit(A, xd, nd, q.ci, q.sbits));
      } else {
      for (int a = 0; a < 3; ++a) {
        G dd = static_cast<G>(INFINITY);
        if (q.d[a] > G(0)) dd = (wall<G>(A, q.ci[a] + 1) - q.x[a]) / q.d[a];
        else if (q.d[a] < G(0)) dd = (wall<G>(A, q.ci[a]) - q.x[a]) / q.d[a];
        q.dist[a] = dd;
        smin = dd < smin ? dd : smin;
      }
      }
      q.smin = smin;
      q.s = smin > G(0) ? smin : G(0);
      q.Dexit = q.D + q.s;
      q.have_exit = true;
      if (!(smin < static_cast<G>(INFINITY))) {  // NaN or zero direction: no wall ahead
        t.bad = true;
        pid = -1;
        continue;
      }
      line_event = q.k < A.L && static_cast<G>(1.0 - q.lamL * nxt.inv_lam) <= q.Dexit;
    }
    if (line_event) {
      const LineRec lr = nxt;
      const int64_t c = SPH ? q.ci[0] + (int64_t)A.sph_nr * (q.ci[1] + (int64_t)A.sph_nt * q.ci[2])
                            : q.ci[0] + (int64_t)A.n * (q.ci[1] + (int64_t)A.n * q.ci[2]);
      const int64_t row = !OCT ? c
          : A.sub_slices ? c - A.sub_c0
          : (q.ci[0] - A.lo[0]) + (int64_t)A.half * ((q.ci[1] - A.lo[1]) + (int64_t)A.half * (q.ci[2] - A.lo[2]));
      const int k = q.k;
      t.checks++;
      // the cell's scale is loaded for every lane, so that the opacity
      // loads of both kinds of line are in flight before the first use
      const float ts = A.tau_scale[c];
      double tct = 0.0, fc = 1.0;
      const int tr = lr.trans;
      if (tr >= 0) {
        tct = A.tau_ct[c * A.T + tr];
        if (A.fcorr_ct) fc = A.fcorr_ct[c * A.T + tr];
      }
      const double tau = tr >= 0 ? tct : static_cast<double>(lr.tau0) * static_cast<double>(ts);
      // the next line's record, and this line's wavelength, are loaded
      // before the estimator atomic: a later wait for them then need not
      // wait for the atomic as well
      q.k = k + 1;
      nxt = line_rec(A, k + 1);
      if (tau > kTauMin) {
        t.inter++;
        const double lam_k = A.lam[k];
        // the continuum up to the resonance, then the line
        if constexpr (PI) pi_move<G>(A, q, c, 1.0 - q.lamL / lam_k, t);
        const double dN = q.w * (-expm1(-tau));
        q.wabs += dN;
        q.w = q.w * exp(-tau);
        if (A.gdirect) {
          if (tr >= 0) atomicAdd(A.gdirect + c * A.T + tr, dN / fc);
        } else {
          atomicAdd(A.est + row * A.L + k, dN / fc);
          if (A.touched) A.touched[row] = 1;
        }
        if (q.w * q.lam_e < (kKillFrac * q.w0) * lam_k) {
          t.w_kill += q.w;
          t.killed++;
          if (A.pk_out) put_record<G, PI>(A.pk_out + kPkFields * (pid - A.first), q, 0.0, q.w);
          stop = true;
        }
      }
    }
    if (stop) {
      t.w_abs += q.wabs;
      pid = -1;
    }
  }

  // ---- per-wave reduction of the tallies, one atomic per wave and field
  double v[11] = {t.w_emit, t.w_esc, t.w_kill, t.w_abs, (double)t.inter, (double)t.checks,
                  (double)t.cross, (double)t.escaped, (double)t.killed, t.e_esc, t.w_pi};
#pragma unroll
  for (int f = 0; f < (PI ? 11 : 10); ++f) {
    double s = wave_sum(v[f]);
    if (lane == 0 && s != 0.0) atomicAdd(A.stats + f, s);
  }
  // packets with an id beyond the sampling plan or a direction with no wall ahead
  if (__ballot(t.bad) != 0ull && lane == 0) A.stats[EXTRASS_STATS - 2] = 1.0;
  // octant mode: a queue was full and packets were lost
  if (__ballot(t.overflow) != 0ull && lane == 0) A.stats[EXTRASS_STAT_QUEUE_FULL] = 1.0;
}

template <class G, bool RAYS, bool PI, bool SPH, bool OCT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_transport(TArgs A) {
  transport_body<G, RAYS, PI, SPH, OCT>(A);
}

// The spherical grid's exit search (three surfaces of each kind, square
// roots, the cone quadratics) needs more registers than three wavefronts per
// SIMD leave: two per SIMD.
template <bool RAYS, bool PI, bool OCT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_transport_sph(TArgs A) {
  transport_body<double, RAYS, PI, true, OCT>(A);
}

}  // namespace
}  // namespace extrass

using namespace extrass;

// Scratch of extrass_transport_noalloc: one array per GPU, held until the
// process ends. Host code never uses its name as an address (on the host it
// is only a stand-in): the device address comes from hipGetSymbolAddress,
// once per device, and is kept in noalloc_ptr.
constexpr size_t kNoAllocBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex noalloc_mutex;
void* noalloc_ptr[kMaxDevices] = {};
}  // namespace

namespace extrass {
// Looks up this device's scratch address once (the device must be current).
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(noalloc_mutex);
  if (noalloc_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) noalloc_ptr[device] = p;
  return e;
}
}  // namespace extrass

struct TransportWs {
  int64_t* start = nullptr;
  LineRec* lines = nullptr;
  unsigned long long* queue = nullptr;
  int32_t* lam_bin = nullptr;
  double* lam_par = nullptr;
  int32_t* chunk_cell = nullptr;
  int64_t nchunk = 0;
  int64_t* tsum = nullptr;  // tile sums of the packet-count scan
  double* sph_cth = nullptr;  // spherical grid: cos of the polar edges
  double* sph_cs = nullptr;   // spherical grid: cos, sin of the azimuthal edges
};

// Spherical-grid fields of A from the grid (none for the cube); false when
// they are invalid.
static bool set_spherical(const extrass_grid* g, TArgs& A) {
  const extrass_spherical* p = g->spherical;
  A.sph_nr = 0;
  if (!p) return true;
  if (p->n_r < 1 || p->n_theta < 1 || p->n_phi < 1 || !p->r_edge || !p->theta_edge ||
      (int64_t)p->n_r * p->n_theta * p->n_phi > INT32_MAX)
    return false;
  A.sph_nr = p->n_r;
  A.sph_nt = p->n_theta;
  A.sph_np = p->n_phi;
  A.sph_r = p->r_edge;
  A.sph_th = p->theta_edge;
  A.sph_dphi = 2.0 * M_PI / p->n_phi;
  return true;
}

static size_t ws_layout(const extrass_grid* g, const extrass_source* s, TransportWs* w, void* ws) {
  const int64_t C = grid_cell_count(g);
  Carver cv(ws, ~size_t(0));
  TransportWs t;
  t.start = cv.take<int64_t>(C + 1);
  t.lines = cv.take<LineRec>(g->n_lines > 0 ? g->n_lines : 1);
  t.queue = cv.take<unsigned long long>(8);
  t.lam_bin = cv.take<int32_t>(lam_bins(g->n_lines));
  t.lam_par = cv.take<double>(2);
  t.nchunk = s->n_packets > 0 ? (s->n_packets + 255) / 256 + 1 : 1;
  t.chunk_cell = cv.take<int32_t>(t.nchunk);
  t.tsum = cv.take<int64_t>((C + kScanTile - 1) / kScanTile + 1);
  if (g->spherical) {
    t.sph_cth = cv.take<double>(g->spherical->n_theta + 1);
    t.sph_cs = cv.take<double>(2 * (g->spherical->n_phi + 1));
  }
  if (w) *w = t;
  return cv.used + 256;
}

// Photoionisation fields of A from the grid's photoion (none when NULL);
// false when they are invalid.
static bool set_photoion(const extrass_grid* g, TArgs& A) {
  const extrass_photoion* p = g->photoion;
  A.pi_M = 0;
  if (!p) return true;
  if (p->n_levels < 1 || p->n_levels > 4096 || !p->lambda_thr || !p->opacity || !p->tally ||
      !(p->length > 0.0))
    return false;
  A.pi_M = p->n_levels;
  A.pi_lam = p->lambda_thr;
  A.pi_opac = p->opacity;
  A.pi_tally = p->tally;
  A.pi_len = p->length;
  return true;
}

// The transport kernel for the geometry precision, emission kind,
// photoionisation and grid (spherical grids: FP64 geometry, no rays).
// Unsplit launches (one kernel per geometry precision, ray and continuum
// option) and streamed visits (OCT: packets handed between subdomains) are
// separate instantiations, so the hand-over code costs the unsplit kernels
// no registers.
static void launch_transport(bool fp32, bool rays, bool pi, bool sph, unsigned blocks,
                             hipStream_t st, const TArgs& A) {
  const dim3 g(blocks), b(kBlock);
  const bool oct = A.oct >= 0;
  if (oct) {  // streamed visits: sampled packets only
    if (sph) {
      if (pi) hipLaunchKernelGGL((k_transport_sph<false, true, true>), g, b, 0, st, A);
      else hipLaunchKernelGGL((k_transport_sph<false, false, true>), g, b, 0, st, A);
    } else if (pi) {
      if (fp32) hipLaunchKernelGGL((k_transport<float, false, true, false, true>), g, b, 0, st, A);
      else hipLaunchKernelGGL((k_transport<double, false, true, false, true>), g, b, 0, st, A);
    } else {
      if (fp32) hipLaunchKernelGGL((k_transport<float, false, false, false, true>), g, b, 0, st, A);
      else hipLaunchKernelGGL((k_transport<double, false, false, false, true>), g, b, 0, st, A);
    }
  } else if (sph) {  // FP64 geometry on the spherical grid
    if (rays && pi) hipLaunchKernelGGL((k_transport_sph<true, true, false>), g, b, 0, st, A);
    else if (rays) hipLaunchKernelGGL((k_transport_sph<true, false, false>), g, b, 0, st, A);
    else if (pi) hipLaunchKernelGGL((k_transport_sph<false, true, false>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_transport_sph<false, false, false>), g, b, 0, st, A);
  } else if (pi) {
    if (rays && fp32) hipLaunchKernelGGL((k_transport<float, true, true, false, false>), g, b, 0, st, A);
    else if (rays) hipLaunchKernelGGL((k_transport<double, true, true, false, false>), g, b, 0, st, A);
    else if (fp32) hipLaunchKernelGGL((k_transport<float, false, true, false, false>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_transport<double, false, true, false, false>), g, b, 0, st, A);
  } else {
    if (rays && fp32) hipLaunchKernelGGL((k_transport<float, true, false, false, false>), g, b, 0, st, A);
    else if (rays) hipLaunchKernelGGL((k_transport<double, true, false, false, false>), g, b, 0, st, A);
    else if (fp32) hipLaunchKernelGGL((k_transport<float, false, false, false, false>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_transport<double, false, false, false, false>), g, b, 0, st, A);
  }
}

extern "C" size_t extrass_transport_workspace(const extrass_grid* g, const extrass_source* s) {
  if (!g || !s || (!g->spherical && g->n <= 0) || s->n_packets < 0) return 0;
  return ws_layout(g, s, nullptr, nullptr);
}

extern "C" int extrass_transport(extrass_handle h, const extrass_grid* g, const extrass_source* s,
                                 double* est, double* stats, double* packets_out, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (!h || !g || !s || !est || !stats || !ws)
    return fail(h, EXTRASS_EINVAL, "extrass_transport: null argument");
  if (!g->spherical && (g->n <= 0 || g->n > 1024 || !(g->beta_max > 0.0)))
    return fail(h, EXTRASS_EINVAL, "extrass_transport: bad grid size");
  if (g->n_lines < 0) return fail(h, EXTRASS_EINVAL, "extrass_transport: bad line count");
  if (g->n_lines > 0 && (!g->line_lambda || !g->line_tau0))
    return fail(h, EXTRASS_EINVAL, "extrass_transport: missing line arrays");
  if (!g->tau_scale) return fail(h, EXTRASS_EINVAL, "extrass_transport: tau_scale is NULL");
  if (g->tau_ct && (!g->line_trans || g->n_trans <= 0))
    return fail(h, EXTRASS_EINVAL, "extrass_transport: tau_ct needs line_trans and n_trans");
  if (s->n_packets < 0 || s->first_packet < 0)
    return fail(h, EXTRASS_EINVAL, "extrass_transport: bad packet range");
  const extrass_rays* rays = s->rays;
  if (rays && (s->explicit_packets || rays->n_theta < 1 || rays->n_phi < 1 ||
               rays->n_theta > 4096 || rays->n_phi > 4096 || rays->n_bins < 0 ||
               (rays->n_bins > 0 && (!rays->bin_lambda || !rays->bin_photons))))
    return fail(h, EXTRASS_EINVAL, "extrass_transport: bad deterministic rays");
  if (!s->explicit_packets && !rays && (!g->cell_packets || !g->cell_photons))
    return fail(h, EXTRASS_EINVAL, "extrass_transport: sampled mode needs cell_packets/photons");
  TArgs A{};
  if (!set_photoion(g, A)) return fail(h, EXTRASS_EINVAL, "extrass_transport: bad photoion");
  if (!set_spherical(g, A)) return fail(h, EXTRASS_EINVAL, "extrass_transport: bad spherical grid");
  TransportWs tw;
  const size_t need = ws_layout(g, s, &tw, ws);
  if (ws_bytes < need) return fail(h, EXTRASS_ENOSPACE, "extrass_transport: workspace too small");
  int64_t* start = tw.start;
  unsigned long long* queue = tw.queue;

  hipStream_t st = static_cast<hipStream_t>(stream);
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  const int64_t C = grid_cell_count(g);
  const int L = g->n_lines;

  const int has_ct = (g->tau_ct && g->line_trans) ? 1 : 0;
  hipLaunchKernelGGL(k_prep, dim3(64), dim3(256), 0, st, g->line_lambda, g->line_tau0,
                     g->line_trans, has_ct, g->n_trans, tw.lines, L, stats, queue);
  if (L > 0)
    hipLaunchKernelGGL(k_check_lines, dim3(64), dim3(256), 0, st, g->line_lambda, g->line_trans,
                       has_ct, g->n_trans, L, stats);
  hipLaunchKernelGGL(k_lambin, dim3(64), dim3(256), 0, st, g->line_lambda, L, lam_bins(L),
                     tw.lam_bin, tw.lam_par);
  if (!s->explicit_packets && !rays) {
    scan_counts(st, g->cell_packets, C, g->n, -1, tw.tsum, start);
    const int64_t b2 = std::min<int64_t>((tw.nchunk + 255) / 256, 4096);
    hipLaunchKernelGGL(k_chunk_cells, dim3((unsigned)std::max<int64_t>(b2, 1)), dim3(256), 0, st,
                       start, C, s->first_packet, tw.nchunk, tw.chunk_cell);
  }
  const int64_t n_est = C * (int64_t)L;
  if (n_est > 0) {
    int64_t blocks = (n_est / 2 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, est, n_est);
  }
  EXTRASS_HIP_TRY(h, hipGetLastError());
  if (s->n_packets == 0) return EXTRASS_OK;

  A.n = g->spherical ? 1 : g->n;
  A.beta = g->spherical ? 1.0 : g->beta_max;
  A.h = 2.0 * A.beta / A.n;
  A.tau_scale = g->tau_scale;
  A.cell_photons = g->cell_photons;
  A.cell_packets = g->cell_packets;
  A.L = L;
  A.lam = g->line_lambda;
  A.lines = tw.lines;
  A.T = g->n_trans;
  A.tau_ct = g->tau_ct;
  A.fcorr_ct = g->fcorr_ct;
  A.seed = s->seed;
  A.iteration = (uint32_t)s->iteration;
  A.first = s->first_packet;
  A.count = s->n_packets;
  A.lam_lo = s->lambda_lo;
  A.lam_hi = s->lambda_hi;
  A.explicit_pk = s->explicit_packets;
  A.start = start;
  A.lam_bin = tw.lam_bin;
  A.lam_par = tw.lam_par;
  A.nbin = lam_bins(L);
  A.chunk_cell = (s->explicit_packets || rays) ? nullptr : tw.chunk_cell;
  if (g->spherical) {
    const int m = std::max(A.sph_nt, A.sph_np) + 1;
    hipLaunchKernelGGL(k_sph_trig, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                       A.sph_th, A.sph_nt, A.sph_np, tw.sph_cth, tw.sph_cs);
    A.sph_cth = tw.sph_cth;
    A.sph_cs = tw.sph_cs;
  }
  if (rays) {
    A.ray_lam = rays->bin_lambda;
    A.ray_ph = rays->n_bins > 0 ? rays->bin_photons : nullptr;
    A.ray_B = rays->n_bins;
    A.ray_nt = rays->n_theta;
    A.ray_np = rays->n_phi;
    if (rays->n_bins == 0) return EXTRASS_OK;  // no bins: no rays
  }
  A.nchunk = tw.nchunk;
  A.C = C;
  A.est = est;
  A.stats = stats;
  A.pk_out = packets_out;
  A.queue = queue;
  A.oct = -1;

  // enough waves to fill every CU several times over, never more than needed
  int64_t blocks = (int64_t)h->num_cus * 8;
  const int64_t max_blocks = (s->n_packets + kBlock - 1) / kBlock;
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  launch_transport(s->geometry_fp32 != 0, rays != nullptr, A.pi_M > 0, A.sph_nr > 0, (unsigned)blocks,
                   st, A);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}

extern "C" int extrass_transport_noalloc(extrass_handle h, const extrass_grid* g,
                                         const extrass_source* s, double* est, double* stats,
                                         double* packets_out, void* stream) {
  if (!h || !g || !s) return fail(h, EXTRASS_EINVAL, "extrass_transport_noalloc: null argument");
  if (h->device < 0 || h->device >= kMaxDevices)
    return fail(h, EXTRASS_EINVAL, "extrass_transport_noalloc: device index");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    ws = noalloc_ptr[h->device];
  }
  if (!ws) return fail(h, EXTRASS_EHIP, "extrass_transport_noalloc: scratch not set up");
  if ((!g->spherical && g->n <= 0) || s->n_packets < 0 ||
      extrass_transport_workspace(g, s) > kNoAllocBytes)
    return fail(h, EXTRASS_ENOSPACE,
                "extrass_transport_noalloc: the problem needs more than the 16 MiB scratch");
  return extrass_transport(h, g, s, est, stats, packets_out, ws, kNoAllocBytes, stream);
}

// ---- streamed transport over velocity octants --------------------------------

namespace {
// Subdomains of the streamed transport: the cube's 8 velocity octants, or a
// spherical grid's n_domains equal ranges of phi (contiguous cells). Both are
// convex, so a straight ray enters each at most once.
struct Domains {
  int n = 8;         // subdomains
  int64_t Co = 0;    // cells per subdomain
  int slices = 0;    // spherical grid: phi slices per subdomain (0: octants)
  int rounds = 5;    // passes over the subdomains that drain every queue
};

Domains domains_of(const extrass_grid* g) {
  Domains d;
  if (g->spherical) {
    d.n = g->spherical->n_domains;
    d.slices = d.n > 0 ? g->spherical->n_phi / d.n : 0;
    d.Co = d.n > 0 ? grid_cell_count(g) / d.n : 0;
    d.rounds = d.n + 1;
  } else {
    const int64_t half = g->n / 2;
    d.Co = half * half * half;
  }
  return d;
}

struct StreamWs {
  int64_t* start;
  LineRec* lines;
  unsigned long long* counters;  // [0] packet pool, [1..n] queue tails, [n + 1] map flag
  int64_t* visit;                // [0] packets of the current visit, [1] its first queued
                                 // record, [2..n + 1] records of each queue already resumed
  int64_t* ostart;               // octants: 8 x (Co + 1)
  QPk* queues;                   // n x qcap
  uint8_t* touched;              // [Co]
  int64_t* tsum;                 // tile sums of the packet-count scans
  int32_t* lam_bin;              // [lam_bins(L)]
  double* lam_par;               // [2]
  double* sph_cth;               // spherical grid: cos of the polar edges
  double* sph_cs;                // spherical grid: cos, sin of the azimuthal edges
  size_t need;
};

StreamWs stream_layout(const extrass_grid* g, int64_t qcap, void* ws) {
  const int64_t C = grid_cell_count(g);
  const Domains dm = domains_of(g);
  const int64_t Co = dm.Co;
  Carver cv(ws, ~size_t(0));
  StreamWs w{};
  w.start = cv.take<int64_t>(C + 1);
  w.lines = cv.take<LineRec>(g->n_lines > 0 ? g->n_lines : 1);
  w.counters = cv.take<unsigned long long>(dm.n + 8);
  w.visit = cv.take<int64_t>(dm.n + 2);
  if (!dm.slices) w.ostart = cv.take<int64_t>(8 * (Co + 1));
  w.queues = cv.take<QPk>((size_t)(dm.n * (qcap > 0 ? qcap : 1)));
  w.touched = cv.take<uint8_t>(Co);
  w.tsum = cv.take<int64_t>((C + kScanTile - 1) / kScanTile + 1);
  w.lam_bin = cv.take<int32_t>(lam_bins(g->n_lines));
  w.lam_par = cv.take<double>(2);
  if (g->spherical) {
    w.sph_cth = cv.take<double>(g->spherical->n_theta + 1);
    w.sph_cs = cv.take<double>(2 * (g->spherical->n_phi + 1));
  }
  w.need = cv.used + 256;
  return w;
}

void zero_doubles(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n / 2 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}
}  // namespace

// A grid the streamed transport can split: an even cube, or a spherical grid
// whose n_phi slices divide into n_domains >= 2 equal subdomains.
static bool streamable(const extrass_grid* g) {
  if (!grid_shape_ok(g)) return false;
  if (g->spherical)
    return g->spherical->n_domains >= 2 && g->spherical->n_phi % g->spherical->n_domains == 0;
  return (g->n & 1) == 0;
}

extern "C" size_t extrass_transport_streamed_workspace(const extrass_grid* g, int64_t queue_capacity) {
  if (!g || !streamable(g) || queue_capacity < 0) return 0;
  return stream_layout(g, queue_capacity, nullptr).need;
}

extern "C" int extrass_transport_streamed(extrass_handle h, const extrass_grid* g,
                                          const extrass_source* s, extrass_atom_handle atom,
                                          const double* pops, double t_exp, double* est_octant,
                                          double* est_global, double* gamma_pe, double* stats,
                                          int64_t queue_capacity, void* ws, size_t ws_bytes,
                                          void* stream) {
  if (!h || !g || !s || !stats || !ws)
    return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: null argument");
  // without an octant table the rates are summed directly per interaction
  const bool direct = est_octant == nullptr;
  if (direct && (!atom || est_global || !g->tau_ct || !g->line_trans ||
                 g->n_trans != (atom ? atom->T : -1)))
    return fail(h, EXTRASS_EINVAL,
                "extrass_transport_streamed: without est_octant, rates need the atom, the grid's "
                "transition opacities and no est_global");
  if (!streamable(g) || g->n_lines <= 0 || !g->line_lambda || !g->line_tau0 || !g->tau_scale ||
      !g->cell_packets || !g->cell_photons)
    return fail(h, EXTRASS_EINVAL,
                "extrass_transport_streamed: bad grid (an even cube, or n_domains dividing n_phi)");
  if (g->tau_ct && (!g->line_trans || g->n_trans <= 0))
    return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: tau_ct needs line_trans and n_trans");
  if (s->explicit_packets || s->rays || s->first_packet != 0 || s->n_packets < 0)
    return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: whole sampling plan only");
  if (atom && (!pops || !gamma_pe || !(t_exp > 0.0)))
    return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: rates need pops, gamma_pe, t_exp");
  if (direct && atom->N > 8192)  // a cell's level reciprocals are staged in 64 KB of LDS
    return fail(h, EXTRASS_EUNSUPPORTED, "extrass_transport_streamed: more than 8192 levels");
  if (atom && atom->maxLine >= g->n_lines)
    return fail(h, EXTRASS_EINVAL,
                "extrass_transport_streamed: a transition's line index is beyond the grid's lines");
  const CellVolume cell_volume = grid_volumes(g, atom ? t_exp : 1.0);
  if (queue_capacity <= 0) return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: queue capacity");
  TArgs A{};
  if (!set_photoion(g, A)) return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: bad photoion");
  if (!set_spherical(g, A)) return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: bad spherical grid");
  StreamWs w = stream_layout(g, queue_capacity, ws);
  if (ws_bytes < w.need) return fail(h, EXTRASS_ENOSPACE, "extrass_transport_streamed: workspace too small");

  hipStream_t st = static_cast<hipStream_t>(stream);
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  const Domains dm = domains_of(g);
  const int ND = dm.n;
  const int n = g->spherical ? 1 : g->n, half = n / 2, L = g->n_lines;
  const int64_t C = grid_cell_count(g), Co = dm.Co;

  const int has_ct = (g->tau_ct && g->line_trans) ? 1 : 0;
  hipLaunchKernelGGL(k_prep, dim3(64), dim3(256), 0, st, g->line_lambda, g->line_tau0,
                     g->line_trans, has_ct, g->n_trans, w.lines, L, stats, w.counters);
  hipLaunchKernelGGL(k_check_lines, dim3(64), dim3(256), 0, st, g->line_lambda, g->line_trans,
                     has_ct, g->n_trans, L, stats);
  scan_counts(st, g->cell_packets, C, n, -1, w.tsum, w.start);
  hipLaunchKernelGGL(k_lambin, dim3(64), dim3(256), 0, st, g->line_lambda, L, lam_bins(L),
                     w.lam_bin, w.lam_par);
  if (!dm.slices)
    for (int o = 0; o < 8; ++o)
      scan_counts(st, g->cell_packets, Co, n, o, w.tsum, w.ostart + o * (Co + 1));
  if (g->spherical) {
    const int m = std::max(A.sph_nt, A.sph_np) + 1;
    hipLaunchKernelGGL(k_sph_trig, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                       A.sph_th, A.sph_nt, A.sph_np, w.sph_cth, w.sph_cs);
    A.sph_cth = w.sph_cth;
    A.sph_cs = w.sph_cs;
  }
  hipLaunchKernelGGL(k_reset_u64, dim3(1), dim3(256), 0, st, w.counters, ND + 8);
  hipLaunchKernelGGL(k_reset_u64, dim3(1), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long*>(w.visit), ND + 2);
  if (atom) zero_doubles(gamma_pe, C * (int64_t)atom->T, st);
  if (est_global) zero_doubles(est_global, C * (int64_t)L, st);
  if (direct) {
    unsigned long long* flag = w.counters + ND + 1;  // zeroed with the counters above
    hipLaunchKernelGGL(k_check_map, dim3(16), dim3(256), 0, st, g->line_trans, L, atom->d.o_line,
                       atom->T, flag);
    unsigned long long bad = 0;
    EXTRASS_HIP_TRY(h, hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st));
    EXTRASS_HIP_TRY(h, hipStreamSynchronize(st));
    if (bad != 0)
      return fail(h, EXTRASS_EINVAL,
                  "extrass_transport_streamed: grid line_trans is not the inverse of the atom's lines");
  } else {
    // the octant table stays zero between visits (each visit's flush clears its rows)
    zero_doubles(est_octant, Co * (int64_t)L, st);
    EXTRASS_HIP_TRY(h, hipMemsetAsync(w.touched, 0, (size_t)Co, st));
  }
  EXTRASS_HIP_TRY(h, hipGetLastError());

  // packets each subdomain emits, and the plan's total
  std::vector<int64_t> n_emit(ND, 0);
  if (dm.slices) {  // contiguous cells: differences of the global prefix
    std::vector<int64_t> edge(ND + 1, 0);
    for (int o = 0; o <= ND; ++o)
      EXTRASS_HIP_TRY(h, hipMemcpyAsync(&edge[o], w.start + o * Co, sizeof(int64_t),
                                        hipMemcpyDeviceToHost, st));
    EXTRASS_HIP_TRY(h, hipStreamSynchronize(st));
    for (int o = 0; o < ND; ++o) n_emit[o] = edge[o + 1] - edge[o];
  } else {
    for (int o = 0; o < 8; ++o)
      EXTRASS_HIP_TRY(h, hipMemcpyAsync(&n_emit[o], w.ostart + o * (Co + 1) + Co, sizeof(int64_t),
                                        hipMemcpyDeviceToHost, st));
    EXTRASS_HIP_TRY(h, hipStreamSynchronize(st));
  }
  int64_t total = 0;
  for (int o = 0; o < ND; ++o) total += n_emit[o];
  if (total != s->n_packets)
    return fail(h, EXTRASS_EINVAL, "extrass_transport_streamed: n_packets differs from the plan");

  A.n = n;
  A.beta = g->spherical ? 1.0 : g->beta_max;
  A.h = 2.0 * A.beta / n;
  A.tau_scale = g->tau_scale;
  A.cell_photons = g->cell_photons;
  A.cell_packets = g->cell_packets;
  A.L = L;
  A.lam = g->line_lambda;
  A.lines = w.lines;
  A.T = g->n_trans;
  A.tau_ct = g->tau_ct;
  A.fcorr_ct = g->fcorr_ct;
  A.seed = s->seed;
  A.iteration = (uint32_t)s->iteration;
  A.first = 0;
  A.lam_lo = s->lambda_lo;
  A.lam_hi = s->lambda_hi;
  A.explicit_pk = nullptr;
  A.start = w.start;
  A.lam_bin = w.lam_bin;
  A.lam_par = w.lam_par;
  A.nbin = lam_bins(L);
  A.chunk_cell = nullptr;
  A.C = C;
  A.est = est_octant;
  A.stats = stats;
  A.pk_out = nullptr;
  A.queue = w.counters;
  A.half = half;
  A.sub_slices = dm.slices;
  A.qbase = w.queues;
  A.qtail = w.counters + 1;
  A.qcap = queue_capacity;
  A.touched = direct ? nullptr : w.touched;
  A.gdirect = direct ? gamma_pe : nullptr;

  std::vector<int64_t> head(ND, 0);
  std::vector<unsigned long long> tail(ND, 0);
  // A ray enters each convex subdomain at most once: the cube's octants take
  // at most 4 rounds, a spherical grid's phi ranges at most n_domains. Rounds
  // alternate their direction: phi along a straight ray is monotonic, so a
  // packet moving towards lower phi ranges is handed on within a backward
  // round instead of waiting one round per range (a visit costs about 1 ms
  // however few packets it resumes). Each visit learns its size on the
  // device (k_visit_begin), so the host waits once per round, to see whether
  // any packet is still queued, not before every visit.
  // launch size of a later round's visit: the packets queued for it when the
  // round began, or an equal share of all those queued, whichever is more
  // (packets handed over during the round add to it; the kernel takes every
  // packet whatever its size)
  std::vector<int64_t> queued_at(ND, 0);
  int64_t queued_all = 0;
  for (int round = 0; round < dm.rounds; ++round) {
    for (int v = 0; v < ND; ++v) {
      const int o = (round & 1) ? ND - 1 - v : v;
      const int64_t ne = round == 0 ? n_emit[o] : 0;
      const int64_t expect = round == 0 ? ne + queued_all
                                        : std::max<int64_t>(queued_at[o], queued_all / ND);
      const int64_t blocks = std::max<int64_t>(
          1, std::min<int64_t>((int64_t)h->num_cus * 8, (expect + kBlock - 1) / kBlock));
      hipLaunchKernelGGL(k_visit_begin, dim3(1), dim3(64), 0, st, o, ne, (int64_t)queue_capacity,
                         w.counters, w.visit);
      A.oct = o;
      A.lo[0] = (o & 1) ? half : 0;
      A.lo[1] = (o & 2) ? half : 0;
      A.lo[2] = (o & 4) ? half : 0;
      A.ostart = dm.slices ? nullptr : w.ostart + o * (Co + 1);
      A.sub_c0 = dm.slices ? (int64_t)o * Co : 0;
      A.n_emit = ne;
      A.visit = w.visit;
      launch_transport(s->geometry_fp32 != 0, false, A.pi_M > 0, g->spherical != nullptr,
                       (unsigned)blocks, st, A);
      EXTRASS_HIP_TRY(h, hipGetLastError());
      if (!direct)
        hipLaunchKernelGGL(k_octant_flush, dim3((unsigned)Co), dim3(256), 0, st, est_octant,
                           w.touched, n, o, dm.slices ? (int64_t)o * Co : (int64_t)-1, L,
                           atom ? atom->N : 0, atom ? atom->T : 0,
                           atom ? atom->d.o_lo : nullptr, atom ? atom->d.o_line : nullptr, pops,
                           cell_volume, atom ? gamma_pe : nullptr, est_global);
      EXTRASS_HIP_TRY(h, hipGetLastError());
    }
    EXTRASS_HIP_TRY(h, hipMemcpyAsync(tail.data(), w.counters + 1, ND * sizeof(unsigned long long),
                                      hipMemcpyDeviceToHost, st));
    EXTRASS_HIP_TRY(h, hipMemcpyAsync(head.data(), w.visit + 2, ND * sizeof(int64_t),
                                      hipMemcpyDeviceToHost, st));
    EXTRASS_HIP_TRY(h, hipStreamSynchronize(st));
    queued_all = 0;
    for (int o = 0; o < ND; ++o) {
      queued_at[o] = std::min<int64_t>((int64_t)tail[o], queue_capacity) - head[o];
      queued_all += queued_at[o];
    }
    if (queued_all == 0) break;
  }
  double full = 0.0;
  EXTRASS_HIP_TRY(h, hipMemcpyAsync(tail.data(), w.counters + 1, ND * sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, st));
  EXTRASS_HIP_TRY(h, hipMemcpyAsync(head.data(), w.visit + 2, ND * sizeof(int64_t),
                                    hipMemcpyDeviceToHost, st));
  EXTRASS_HIP_TRY(h, hipMemcpyAsync(&full, stats + EXTRASS_STAT_QUEUE_FULL, sizeof(double),
                                    hipMemcpyDeviceToHost, st));
  EXTRASS_HIP_TRY(h, hipStreamSynchronize(st));
  if (full != 0.0)
    return fail(h, EXTRASS_ENOSPACE, "extrass_transport_streamed: a subdomain queue overflowed");
  for (int o = 0; o < ND; ++o)
    if ((int64_t)tail[o] != head[o])
      return fail(h, EXTRASS_EHIP, "extrass_transport_streamed: packets left in a queue");
  if (direct) {
    const int64_t blocks = std::min<int64_t>(C, 16384);
    hipLaunchKernelGGL(k_rates_direct, dim3((unsigned)blocks), dim3(256),
                       (size_t)atom->N * sizeof(double), st, C, atom->N, atom->T, atom->d.o_lo, pops,
                       cell_volume, gamma_pe);
    EXTRASS_HIP_TRY(h, hipGetLastError());
  }
  return EXTRASS_OK;
}
