// Batched NLTE solve: one element with three ion stages per cell under frozen
// rates (Sec. 2.2; the rate model is stated in extrass.h).
//
// Structure used: the excited levels of a stage exchange population only with
// the levels of that stage and with the next stage's ground state (ionisation
// into it, recombination out of it). Block z of a cell holds the states
//   [excited levels 1..L_z-1 of stage z] [ground of z] [ground of z+1]
// (B = L_z + 1; B = L_z for the top stage). Eliminating the excited levels of
// every block is the state reduction (Grassmann-Taksar-Heyman) of the full
// matrix in an order that skips only exact zeros; the ground states left form
// a birth-death chain, solved in closed form, and back-substitution gives the
// excited levels.
//
// Kernels per chunk of cells:
//  k_assemble     one work-group per block: rates from the Philox draws into a
//                 row-major B x B matrix (FP64, and FP32 for the FP32 factor)
//  k_factor<T,NB> persistent work-groups take blocks, largest first, and run the
//                 blocked reduction; per panel of NB eliminated states:
//                 (a) row sums of the panel rows over the trailing states;
//                 (b) the NB x NB diagonal block reduced in LDS, each pivot the
//                     sum of its row's remaining off-diagonal rates;
//                 (c) panel rows (trailing columns) and panel columns (trailing
//                     rows) brought to their elimination time by unit-triangular
//                     recurrences, one column or row per thread;
//                 (d) trailing update A_TT += C diag(1/S) R on matrix cores
//                     (MFMA 16x16x4 in T), one 32 x 32 tile per wavefront step;
//                     panels go in groups of 32 states: each panel's rows and
//                     columns take the update of the group's earlier panels
//                     before its steps (a)-(c), and the rest of the trailing
//                     matrix takes one update of the whole group (rank up to
//                     32), read and written once per group (groups of 48 and
//                     64 states measured the same: the wider update re-reads
//                     its operands per 32 x 32 tile).
//                 Every term is a product of non-negative rates: there is no
//                 subtraction, so populations down to 1e-30 keep their accuracy.
//  k_chain        per cell: the ground-state chain
//  k_backsub<T>   per block: excited-level populations (or corrections)
//  k_residual, k_forward<T>   iterative refinement of the FP32 factorisation:
//                 FP64 residual from the FP64 matrix, correction solved with
//                 the FP32 factors in FP64 arithmetic
//  k_normalise    per cell: sum to 1, status
//
// Factored block layout (row-major, leading dimension B): for an eliminated
// state i, entries right of the diagonal hold row i at its elimination time,
// entries below hold column i at that time divided by the pivot S_i; the
// trailing 2 x 2 of the ground states holds the reduced rates between them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "philox.hpp"

namespace extrass {
namespace {

constexpr double kBoltz = 1.380649e-16;  // erg/K
constexpr int kThreads = 256;
constexpr int kMaxLevels = 1023;
constexpr int kMaxB = kMaxLevels + 1;
// states eliminated per group of panels (column factors kept for one update);
// a panel wider than the group is a group of its own
constexpr int kGroup = 32;
// rows of column factors per resident work-group: the widest group
constexpr int kCtRows = kGroup > 64 ? kGroup : 64;
constexpr uint64_t kPhiloxStream = 6;

struct Blk {
  int64_t a;     // offset of the block matrix (elements) in the matrix arena
  int64_t v;     // offset of the block's per-state vectors
  int32_t cell;  // cell index within the chunk
  int32_t z;     // ion stage
  int32_t B;     // states in the block
  int32_t L;     // levels of the stage
};

struct Args {
  const Blk* blk;
  int nblk;
  int ncell;             // cells in the chunk
  int64_t c0;            // first cell of the chunk
  uint64_t seed;
  const int32_t* L;      // [C*3]
  const int64_t* pop;    // [C+1] first population of each cell (all cells)
  const double* T_e;
  const double* n_e;
  const double* gion;
  const double* gpe_tab;  // [n_gpe] photoexcitation rates, ascending
  int64_t n_gpe;
  double alpha0_0, alpha0_1;
  double* A64;
  float* A32;
  double* S;             // pivots, per block state
  double* rowsum;        // FP64 row sums of the assembled matrix (refinement)
  double* bvec;          // right-hand side per block state (refinement)
  double* scale;         // [nblk] power of two applied to the FP32 matrix (refinement)
  double* red;           // [nblk*2] reduced rates ground z -> z+1, z+1 -> z
  double* rb;            // [nblk*2] reduced right-hand side at the two grounds
  const int32_t* cell_blk;  // [ncell*3] block of each stage, -1 if absent
  double* gval;          // [ncell*3] ground-state values (populations or corrections)
  unsigned long long* maxrel;  // [ncell] bits of max |correction / population|
  void* ct;              // column factors of one group of panels per resident work-group
  int maxB;              // largest block of the problem (LDS of the assembly)
  int ldct;
  unsigned int* queue;
  double* pops;
  int32_t* status;
};

// Level of block position p (-1 for the next stage's ground).
__device__ __forceinline__ int pos_level(int p, int L) {
  return p < L - 1 ? p + 1 : (p == L - 1 ? 0 : -1);
}

// Population index of block position p within the cell.
__device__ __forceinline__ int64_t pos_index(const Args& A, int64_t c, int z, int p, int L) {
  const int32_t* Lc = A.L + 3 * c;
  int64_t base = A.pop[c];
  for (int k = 0; k < z; ++k) base += Lc[k];
  const int lv = pos_level(p, L);
  return lv >= 0 ? base + lv : base + L;  // next ground = level 0 of stage z+1
}

// ---- assembly -------------------------------------------------------------
// Rates of the pair of block positions p != q, both directions: v = p -> q,
// vt = q -> p. Two levels share one Philox draw (keyed by the lower and the
// higher level index); the next stage's ground pairs with every level through
// ionisation (level -> next ground) and recombination (next ground -> level).
__device__ __forceinline__ void pair_rates(const Args& A, int64_t c, int z, int L, int p, int q,
                                           const double* gs, const double* Es, double kT,
                                           double ne, double gi, double rec, double gex,
                                           double& v, double& vt) {
  const int lp = pos_level(p, L), lq = pos_level(q, L);
  if (lp >= 0 && lq >= 0) {
    const int l = min(lp, lq), u = max(lp, lq);
    const u64x4 r = philox4x64_10((uint64_t)c, (uint64_t)z, (uint64_t)l, (uint64_t)u, A.seed,
                                  kPhiloxStream);
    const int up = Es[u] >= Es[l] ? u : l, lo = up == u ? l : u;
    const bool rad = unit53(r.v[0]) < 0.2;
    const double Ad = rad ? exp10(-3.0 + 11.0 * unit53(r.v[1])) : 0.0;
    int64_t it = (int64_t)(unit53(r.v[3]) * (double)A.n_gpe);
    it = it < A.n_gpe - 1 ? it : A.n_gpe - 1;
    const double gam = rad ? A.gpe_tab[it] : 0.0;
    const double q10 = exp10(-10.0 + 3.0 * unit53(r.v[2]));
    const double down = Ad + ne * q10 + (gs[lo] / gs[up]) * gam;
    const double upw = ne * q10 * (gs[up] / gs[lo]) * exp(-(Es[up] - Es[lo]) / kT) + gam;
    v = lp == up ? down : upw;
    vt = lp == up ? upw : down;
  } else {
    const int lv = lp >= 0 ? lp : lq;  // the level paired with the next ground
    const double rc = lv == 0 ? rec / 3.0 : rec * (2.0 / 3.0) * gs[lv] / gex;
    v = lp >= 0 ? gi : rc;
    vt = lp >= 0 ? rc : gi;
  }
}

// One work-group per block. The B x B matrix is walked in 64 x 64 tile pairs
// (I <= J): each pair of positions is drawn once, the rates p -> q go straight
// to tile (I, J) and the rates q -> p through LDS, transposed, to tile (J, I),
// so that both stores are coalesced. Row sums (FP32 mode) are accumulated in
// LDS in a fixed tile order.
__global__ __launch_bounds__(kThreads) void k_assemble(Args A, int fp32) {
  extern __shared__ double sm[];
  const Blk bk = A.blk[blockIdx.x];
  const int maxB = A.maxB;
  double* gs = sm;                  // [maxB] statistical weights
  double* Es = sm + maxB;           // [maxB] level energies
  double* racc = sm + 2 * maxB;     // [maxB] row sums
  double* tile = sm + 3 * maxB;     // [64][65] transposed rates of a tile pair
  double* gex_s = tile + 64 * 65;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c = A.c0 + bk.cell;
  const int z = bk.z, L = bk.L, B = bk.B;
  const double T = A.T_e[c], ne = A.n_e[c], kT = kBoltz * T;
  for (int i = tid; i < L; i += kThreads) {
    const u64x4 r = philox4x64_10((uint64_t)c, (uint64_t)z, (uint64_t)i, 1ull << 63, A.seed,
                                  kPhiloxStream);
    gs[i] = 1.0 + floor(9.0 * unit53(r.v[0]));
    Es[i] = i == 0 ? 0.0 : 69.0 * kT * unit53(r.v[1]);
  }
  for (int i = tid; i < B; i += kThreads) racc[i] = 0.0;
  __syncthreads();
  if (wave == 0) {
    double s = 0.0;
    for (int i = 1 + lane; i < L; i += 64) s += gs[i];
    s = wave_sum(s);
    if (lane == 0) *gex_s = s;
  }
  __syncthreads();
  const double gex = *gex_s;
  const double rec = ne * (z == 0 ? A.alpha0_0 : A.alpha0_1) * pow(T / 1e4, -0.8);
  const double gi = z < 2 ? A.gion[2 * c + z] : 0.0;
  double* M64 = A.A64 + bk.a;
  float* M32 = fp32 ? A.A32 + bk.a : nullptr;
  // FP32 copy: scaled by a power of two that brings the largest possible rate
  // of the cell (A <= 1e8, q <= 1e-7, Gamma_PE <= the table's last, g ratio <= 9, ionisation
  // and recombination of either stage) to ~2^100, so that rates ~70 decades
  // below it stay normal. GTH quotients are scale-free; the factor is the same
  // for the blocks of a cell, whose reduced rates meet in the ground-state chain.
  double sc = 1.0;
  if (fp32) {
    const double rec_max = ne * fmax(A.alpha0_0, A.alpha0_1) * pow(T / 1e4, -0.8);
    const double bound = 1e8 + 9.0 * ne * 1e-7 + 9.0 * A.gpe_tab[A.n_gpe - 1] +
                         fmax(A.gion[2 * c], A.gion[2 * c + 1]) +
                         rec_max;
    sc = ldexp(1.0, 100 - ilogb(bound));
    if (tid == 0) A.scale[blockIdx.x] = sc;
  }
  const int nt = (B + 63) >> 6;
  for (int I = 0; I < nt; ++I)
    for (int J = I; J < nt; ++J) {
      const int p0 = 64 * I, q0 = 64 * J;
      const int q = q0 + lane;
      // rows p of tile I against columns q of tile J (p < q on the diagonal tile)
#pragma unroll 1
      for (int pl = wave; pl < 64; pl += 4) {
        const int p = p0 + pl;
        if (p >= B) break;
        double v = 0.0, vt = 0.0;
        if (q < B && (I < J || pl < lane))
          pair_rates(A, c, z, L, p, q, gs, Es, kT, ne, gi, rec, gex, v, vt);
        if (q < B && (I < J || pl <= lane)) {
          M64[(int64_t)p * B + q] = v;
          if (M32) M32[(int64_t)p * B + q] = (float)(v * sc);
        }
        tile[lane * 65 + pl] = vt;
        if (fp32) {
          const double rs = wave_sum(v);
          if (lane == 0) racc[p] += rs;
        }
      }
      __syncthreads();
      // the transposed rates: rows r of tile J, columns of tile I
#pragma unroll 1
      for (int rl = wave; rl < 64; rl += 4) {
        const int rr = q0 + rl, col = p0 + lane;
        if (rr >= B) break;
        // on the diagonal tile only the part below the diagonal comes from here
        const bool mine = col < B && (I < J || lane < rl);
        const double vt = mine ? tile[rl * 65 + lane] : 0.0;
        if (mine) {
          M64[(int64_t)rr * B + col] = vt;
          if (M32) M32[(int64_t)rr * B + col] = (float)(vt * sc);
        }
        if (fp32) {
          const double rs = wave_sum(vt);
          if (lane == 0) racc[rr] += rs;
        }
      }
      __syncthreads();
    }
  if (fp32)
    for (int i = tid; i < B; i += kThreads) A.rowsum[bk.v + i] = racc[i];
}

size_t assemble_lds(const Args& a) { return sizeof(double) * (3 * (size_t)a.maxB + 64 * 65 + 1); }

// ---- matrix-core trailing update -----------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class T> struct Acc;
// Accumulator row of register q in lanes with l/16 = lk (column l%16 in both):
// FP64 16x16x4 interleaves (row lk + 4q), FP32 16x16x4 blocks (row 4 lk + q).
template <> struct Acc<double> {
  typedef d4 type;
  static __device__ __forceinline__ int row(int lk, int q) { return lk + 4 * q; }
  static __device__ __forceinline__ d4 mma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Acc<float> {
  typedef f4 type;
  static __device__ __forceinline__ int row(int lk, int q) { return 4 * lk + q; }
  static __device__ __forceinline__ f4 mma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// M[t][u] += sum_{k < K} Ct(k, t) M[p0 + k][u] for t in [r0, r0 + nr),
// u in [s0, s0 + ns): the rank-K update of a window of the trailing matrix by
// the panel rows p0 .. p0 + K - 1 (at their elimination time) and their
// column factors, Ct(k, t) = ct[k][t - cb.b[k / nb]] (the column factors of
// each panel of nb rows start at that panel's first trailing row). Operand layout
// of the 16x16x4 instructions (lane l): A-operand row l%16, k l/16; B-operand
// column l%16, k l/16; accumulator column l%16, row Acc<T>::row(l/16, q) for
// register q. Rows [K, roundup4(K)) of ct are zero.
struct Bases {
  int b[4];
};

template <class T, int RA = 2>
__device__ void trailing_update(T* M, int B, int p0, int K, int r0, int nr, int s0, int ns,
                                const T* ct, int ldct, int nb, const Bases& cb) {
  typedef typename Acc<T>::type V;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // tiles of 16 RA rows x 32 columns per wavefront
  const int nsr = (nr + 16 * RA - 1) / (16 * RA), nss = (ns + 31) >> 5;
  const int ksteps = (K + 3) >> 2;
  const int lr = lane & 15, lk = lane >> 4;
  for (int tile = wave; tile < nsr * nss; tile += kThreads / 64) {
    const int tr = (tile / nss) * (16 * RA), ts0 = (tile % nss) << 5;
    V acc[RA][2];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = tr + 16 * a + Acc<T>::row(lk, q), c = ts0 + 16 * b + lr;
          acc[a][b][q] = (r < nr && c < ns) ? M[(int64_t)(r0 + r) * B + s0 + c] : T(0);
        }
    for (int ks = 0; ks < ksteps; ++ks) {
      const int k = 4 * ks + lk;
      const int cbk = cb.b[k / nb];
      T av[RA], bv[2];
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        const int r = tr + 16 * a + lr;
        av[a] = r < nr ? ct[(int64_t)k * ldct + (r0 + r - cbk)] : T(0);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int c = ts0 + 16 * b + lr;
        bv[b] = (c < ns && k < K) ? M[(int64_t)(p0 + k) * B + s0 + c] : T(0);
      }
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = Acc<T>::mma(av[a], bv[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = tr + 16 * a + Acc<T>::row(lk, q), c = ts0 + 16 * b + lr;
          if (r < nr && c < ns) M[(int64_t)(r0 + r) * B + s0 + c] = acc[a][b][q];
        }
  }
}

// ---- blocked factorisation --------------------------------------------------
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void k_factor(Args A) {
  __shared__ double D[NB][NB + 1];   // diagonal block: rows (upper) and columns (lower) at
                                     // their elimination time
  __shared__ double U[NB][NB + 1];   // upper part divided by the pivot of its row, lower part
                                     // divided by the pivot of its column
  __shared__ double ts[NB];          // trailing row sums of the panel rows
  __shared__ double Sp[NB];
  __shared__ double inv_s[NB];
  __shared__ int item;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // column factors of a group of kGroup / NB panels for the combined update
  constexpr int P = kGroup / NB > 1 ? kGroup / NB : 1;
  T* ct = reinterpret_cast<T*>(A.ct) + (int64_t)blockIdx.x * kCtRows * A.ldct;
  T* arena = sizeof(T) == 8 ? reinterpret_cast<T*>(A.A64) : reinterpret_cast<T*>(A.A32);
  for (;;) {
    if (tid == 0) item = (int)atomicAdd(A.queue, 1u);
    __syncthreads();
    const int b = item;
    __syncthreads();
    if (b >= A.nblk) break;
    const Blk bk = A.blk[b];
    const int B = bk.B, ne = bk.L - 1;
    T* M = arena + bk.a;
    double* S = A.S + bk.v;
    // One panel of np states from p0: (a)-(c) below; its column factors go
    // to ctp, row t - t0 of each.
    auto panel = [&](int p0, int np, T* ctp) {
      const int t0 = p0 + np;
      // (a) trailing row sums of the panel rows; the diagonal block into LDS
      for (int k = wave; k < np; k += kThreads / 64) {
        double s = 0.0;
        for (int j = t0 + lane; j < B; j += 64) s += (double)M[(int64_t)(p0 + k) * B + j];
        s = wave_sum(s);
        if (lane == 0) ts[k] = s;
      }
      for (int e = tid; e < np * np; e += kThreads) {
        const int r = e / np, q = e - r * np;
        D[r][q] = (double)M[(int64_t)(p0 + r) * B + p0 + q];
      }
      __syncthreads();
      // (b) reduce the diagonal block in one wavefront: its LDS accesses are
      // performed in program order, so the steps need no work-group barrier
      if (wave == 0) {
        for (int i = 0; i < np; ++i) {
          double s = 0.0;
          for (int q = i + 1 + lane; q < np; q += 64) s += D[i][q];
          s = wave_sum(s) + ts[i];
          const double Si = s > 0.0 ? s : NAN;
          if (lane == 0) Sp[i] = Si;
          const double inv = 1.0 / Si;
          const int m = np - 1 - i;
          for (int e = lane; e < m * m; e += 64) {
            const int k = i + 1 + e / m, q = i + 1 + e % m;
            if (k != q) D[k][q] += D[k][i] * D[i][q] * inv;
          }
          for (int k = i + 1 + lane; k < np; k += 64) ts[k] += D[k][i] * ts[i] * inv;
          __asm__ volatile("" ::: "memory");  // step i's stores before step i+1's loads
        }
      }
      __syncthreads();
      for (int e = tid; e < np * np; e += kThreads) {
        const int r = e / np, q = e - r * np;
        U[r][q] = q > r ? D[r][q] / Sp[r] : (q < r ? D[r][q] / Sp[q] : 0.0);
        // factored diagonal block back: rows unscaled, columns divided by the pivot
        if (q != r) M[(int64_t)(p0 + r) * B + p0 + q] = (T)(q > r ? D[r][q] : U[r][q]);
      }
      for (int i = tid; i < np; i += kThreads) {
        S[p0 + i] = Sp[i];
        inv_s[i] = 1.0 / Sp[i];
      }
      __syncthreads();
      // (c) panel rows over the trailing columns: r_i = a_i + sum_{l<i} (D_il/S_l) r_l
      for (int j = t0 + tid; j < B; j += kThreads) {
        // keeps the multiplier loads inside the loop instead of hoisting NB^2/2 of them
        __asm__ volatile("" ::: "memory");
        double r[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) r[i] = i < np ? (double)M[(int64_t)(p0 + i) * B + j] : 0.0;
#pragma unroll
        for (int i = 1; i < NB; ++i) {
          if (i < np) {
            double acc = r[i];
#pragma unroll
            for (int l = 0; l < i; ++l) acc += U[i][l] * r[l];
            r[i] = acc;
          }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (i < np) M[(int64_t)(p0 + i) * B + j] = (T)r[i];
      }
      //     panel columns over the trailing rows: c_i = a_i + sum_{l<i} c_l (D_li/S_l),
      //     stored divided by S_i, also transposed into ct for the update
      for (int t = t0 + tid; t < B; t += kThreads) {
        __asm__ volatile("" ::: "memory");
        double cv[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) cv[i] = i < np ? (double)M[(int64_t)t * B + p0 + i] : 0.0;
#pragma unroll
        for (int i = 1; i < NB; ++i) {
          if (i < np) {
            double acc = cv[i];
#pragma unroll
            for (int l = 0; l < i; ++l) acc += cv[l] * U[l][i];
            cv[i] = acc;
          }
        }
        const int np4 = (np + 3) & ~3;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          if (i < np) {
            const T v = (T)(cv[i] * inv_s[i]);
            M[(int64_t)t * B + p0 + i] = v;
            ctp[(int64_t)i * A.ldct + (t - t0)] = v;
          } else if (i < np4) {
            ctp[(int64_t)i * A.ldct + (t - t0)] = T(0);
          }
        }
      }
      __syncthreads();
    };
    // Panels in groups of kGroup states. Before its steps (a)-(c), a panel's
    // rows and columns (all that those steps read) take the update of the
    // group's earlier panels; after the group, (d) one update of rank up to
    // kGroup brings the rest of the trailing matrix forward by all of them,
    // read and written once per group instead of once per panel.
    for (int g0 = 0; g0 < ne; g0 += P * NB) {
      Bases cb{};
      int K = 0, pj = g0;
#pragma unroll 1
      for (int j = 0; j < P && pj < ne; ++j) {
        const int np = min(NB, ne - pj);
        if (j > 0) {
          trailing_update<T>(M, B, g0, K, pj, np, pj, B - pj, ct, A.ldct, NB, cb);
          trailing_update<T>(M, B, g0, K, pj + np, B - pj - np, pj, np, ct, A.ldct, NB, cb);
          __syncthreads();
        }
        panel(pj, np, ct + (int64_t)j * NB * A.ldct);
        pj += np;
        cb.b[j] = pj;
        K += np;
      }
      // 64 x 32 tiles per wavefront in FP64 (fewer operand loads per entry);
      // in FP32 they cost the kernel its third wavefront per SIMD
      trailing_update<T, sizeof(T) == 8 ? 4 : 2>(M, B, g0, K, pj, B - pj, pj, B - pj, ct, A.ldct,
                                                 NB, cb);
      __syncthreads();
    }
    if (tid == 0 && B == bk.L + 1) {
      A.red[2 * b] = (double)M[(int64_t)(bk.L - 1) * B + bk.L];
      A.red[2 * b + 1] = (double)M[(int64_t)bk.L * B + bk.L - 1];
    }
  }
}

// ---- ground-state chain -----------------------------------------------------
// States g_0..g_{K-1}; g_z -> g_{z+1} at u_z, g_{z+1} -> g_z at d_z (reduced
// rates of block z). Reducing g_0, g_1, ... in turn leaves each pivot equal to
// u_z and carries the right-hand side up unchanged; with x_{K-1} fixed
// (1 for the populations, 0 for a correction), x_z = (x_{z+1} d_z - b_z) / u_z.
__global__ void k_chain(Args A, int rhs) {
  const int cl = blockIdx.x * blockDim.x + threadIdx.x;
  if (cl >= A.ncell) return;
  int bz[3], K = 0;
  for (int z = 0; z < 3; ++z) {
    bz[z] = A.cell_blk[3 * cl + z];
    if (bz[z] >= 0) K = z + 1;
  }
  double bg[3] = {0.0, 0.0, 0.0}, x[3] = {0.0, 0.0, 0.0};
  if (rhs) {
    for (int z = 0; z < K; ++z) bg[z] = A.rb[2 * bz[z]] + (z > 0 ? A.rb[2 * bz[z - 1] + 1] : 0.0);
    for (int z = 0; z + 1 < K; ++z) bg[z + 1] += bg[z];
  }
  x[K - 1] = rhs ? 0.0 : 1.0;
  for (int z = K - 2; z >= 0; --z) {
    const double u = A.red[2 * bz[z]], d = A.red[2 * bz[z] + 1];
    x[z] = (x[z + 1] * d - bg[z]) / u;
  }
  const int64_t c = A.c0 + cl;
  int64_t base = A.pop[c];
  for (int z = 0; z < K; ++z) {
    A.gval[3 * cl + z] = x[z];
    double* p = A.pops + base;
    if (rhs) {
      const double nv = *p + x[z];
      *p = nv;
      const double rel = fabs(x[z]) / fabs(nv);
      atomicMax(A.maxrel + cl, (unsigned long long)__double_as_longlong(rel == rel ? rel : INFINITY));
    } else {
      *p = x[z];
    }
    base += A.L[3 * c + z];
  }
}

// ---- back-substitution: x_k = sum_{j>k} x_j Lc[j][k] - b_k / S_k ----------------
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void k_backsub(Args A, int rhs) {
  __shared__ double xs[kMaxB];
  __shared__ double part[kThreads];
  const Blk bk = A.blk[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int B = bk.B, L = bk.L, ne = L - 1;
  const int64_t c = A.c0 + bk.cell;
  const T* M = (sizeof(T) == 8 ? reinterpret_cast<const T*>(A.A64)
                               : reinterpret_cast<const T*>(A.A32)) + bk.a;
  const double* S = A.S + bk.v;
  if (tid == 0) {
    xs[L - 1] = A.gval[3 * bk.cell + bk.z];
    if (B == L + 1) xs[L] = A.gval[3 * bk.cell + bk.z + 1];
  }
  __syncthreads();
  constexpr int kSlices = kThreads / NB;
  const int kk = tid % NB, slice = tid / NB;
  for (int p0 = ((ne - 1) / NB) * NB; ne > 0 && p0 >= 0; p0 -= NB) {
    const int np = min(NB, ne - p0), t0 = p0 + np;
    double acc = 0.0;
    if (kk < np)
      for (int j = t0 + slice; j < B; j += kSlices)
        acc += xs[j] * (double)M[(int64_t)j * B + p0 + kk];
    part[tid] = acc;
    __syncthreads();
    if (wave == 0) {
      // in-panel recurrence, descending, one wavefront
      for (int k = np - 1; k >= 0; --k) {
        double s = 0.0;
        if (lane == 0)
          for (int sl = 0; sl < kSlices; ++sl) s += part[sl * NB + k];
        const int q = k + 1 + lane;
        double v = q < np ? xs[p0 + q] * (double)M[(int64_t)(p0 + q) * B + p0 + k] : 0.0;
        v = wave_sum(v);
        if (lane == 0) xs[p0 + k] = s + v - (rhs ? A.bvec[bk.v + p0 + k] / S[p0 + k] : 0.0);
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the LDS store is visible
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
  // write the excited levels
  const int64_t base = pos_index(A, c, bk.z, 0, L);  // level 1 of the stage
  for (int p = tid; p < ne; p += kThreads) {
    const double x = xs[p];
    if (rhs) {
      const double nv = A.pops[base + p] + x;
      A.pops[base + p] = nv;
      const double rel = fabs(x) / fabs(nv);
      atomicMax(A.maxrel + bk.cell,
                (unsigned long long)__double_as_longlong(rel == rel ? rel : INFINITY));
    } else {
      A.pops[base + p] = x;
    }
  }
}

// ---- refinement: FP64 residual and forward reduction of the right-hand side ----
// bvec_j = -(sum_i n_i a_ij - n_j rowsum_j) over the block's states (the part of
// the cell's balance that this block's rates carry), times the block's FP32
// scale so that it matches the scaled factors.
__global__ __launch_bounds__(kThreads) void k_residual(Args A) {
  __shared__ double ns[kMaxB];
  const Blk bk = A.blk[blockIdx.x];
  const int tid = threadIdx.x;
  const int B = bk.B, L = bk.L;
  const int64_t c = A.c0 + bk.cell;
  for (int p = tid; p < B; p += kThreads) ns[p] = A.pops[pos_index(A, c, bk.z, p, L)];
  __syncthreads();
  const double* M = A.A64 + bk.a;
  const double sc = A.scale[blockIdx.x];  // the FP32 factors carry this factor
  for (int j = tid; j < B; j += kThreads) {
    double in = 0.0;
    for (int i = 0; i < B; ++i) in += ns[i] * M[(int64_t)i * B + j];
    A.bvec[bk.v + j] = -(in - ns[j] * A.rowsum[bk.v + j]) * sc;
  }
}

template <class T, int NB>
__global__ __launch_bounds__(kThreads) void k_forward(Args A) {
  __shared__ double bs[kMaxB];
  const Blk bk = A.blk[blockIdx.x];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int B = bk.B, L = bk.L, ne = L - 1;
  const T* M = (sizeof(T) == 8 ? reinterpret_cast<const T*>(A.A64)
                               : reinterpret_cast<const T*>(A.A32)) + bk.a;
  const double* S = A.S + bk.v;
  for (int p = tid; p < B; p += kThreads) bs[p] = A.bvec[bk.v + p];
  __syncthreads();
  for (int p0 = 0; p0 < ne; p0 += NB) {
    const int np = min(NB, ne - p0), t0 = p0 + np;
    if (tid < 64) {  // in-panel steps in one wavefront (LDS in program order)
      for (int k = 0; k < np; ++k) {
        const double f = bs[p0 + k] / S[p0 + k];
        const int q = p0 + k + 1 + tid;
        if (q < t0) bs[q] += f * (double)M[(int64_t)(p0 + k) * B + q];
        __asm__ volatile("" ::: "memory");
      }
    }
    __syncthreads();
    for (int j = t0 + tid; j < B; j += kThreads) {
      double acc = bs[j];
      for (int k = 0; k < np; ++k)
        acc += bs[p0 + k] / S[p0 + k] * (double)M[(int64_t)(p0 + k) * B + j];
      bs[j] = acc;
    }
    __syncthreads();
  }
  for (int p = tid; p < B; p += kThreads) A.bvec[bk.v + p] = bs[p];
  if (tid == 0) {
    A.rb[2 * b] = bs[L - 1];
    A.rb[2 * b + 1] = B == L + 1 ? bs[L] : 0.0;
  }
}

// ---- normalisation and status (one wavefront per cell) ------------------------
__global__ __launch_bounds__(kThreads) void k_normalise(Args A, int refined, double tol) {
  const int cl = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (cl >= A.ncell) return;
  const int64_t c = A.c0 + cl;
  const int64_t b0 = A.pop[c], b1 = A.pop[c + 1];
  double s = 0.0, mn = INFINITY;
  for (int64_t i = b0 + lane; i < b1; i += 64) {
    const double v = A.pops[i];
    s += v;
    mn = fmin(mn, v);
  }
  s = wave_sum(s);
  for (int off = 32; off > 0; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off, 64));
  const double inv = 1.0 / s;
  for (int64_t i = b0 + lane; i < b1; i += 64) A.pops[i] *= inv;
  if (lane == 0) {
    int st = 0;
    if (!(mn > 0.0) || !(s < INFINITY)) {
      st = 2;
    } else if (refined) {
      const double rel = __longlong_as_double((long long)A.maxrel[cl]);
      if (!(rel <= tol)) st = 1;
    }
    A.status[c] = st;
  }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_zero_queue(unsigned int* q) { *q = 0u; }

// ---- host planning ------------------------------------------------------------
struct Chunk {
  int64_t c0, c1;
  int64_t blk0, nblk;    // slice of the block table
  int64_t a_elems, v_elems;
};

struct Plan {
  std::vector<Blk> blk;          // all blocks, chunk by chunk, each chunk largest first
  std::vector<int32_t> cell_blk; // [C*3] chunk-local block index
  std::vector<int64_t> pop;      // [C+1]
  std::vector<Chunk> chunks;
  int maxB = 1;
};

int block_states(const int32_t* Lc, int z) {
  return Lc[z] + ((z < 2 && Lc[z + 1] > 0) ? 1 : 0);
}

int64_t round32(int64_t n) { return (n + 31) & ~int64_t(31); }

int64_t cell_matrix_elems(const int32_t* Lc) {
  int64_t e = 0;
  for (int z = 0; z < 3; ++z)
    if (Lc[z] > 0) e += round32((int64_t)block_states(Lc, z) * block_states(Lc, z));
  return e;
}

int64_t cell_vector_elems(const int32_t* Lc) {
  int64_t e = 0;
  for (int z = 0; z < 3; ++z)
    if (Lc[z] > 0) e += round32(block_states(Lc, z));
  return e;
}

struct Layout {
  int panel, per_cu, fp32;
  int64_t G;          // resident work-groups of the factorisation
  int ldct;
  size_t fixed;       // tables + panel scratch + queue
};

size_t arena_bytes(const Layout& y, int64_t a_elems, int64_t v_elems, int64_t nblk, int64_t ncell) {
  size_t s = 0;
  s += carve_bytes<double>(a_elems);
  if (y.fp32) s += carve_bytes<float>(a_elems);
  s += carve_bytes<double>(v_elems) * (y.fp32 ? 3 : 1);
  s += carve_bytes<double>(2 * nblk) * 2;
  if (y.fp32) s += carve_bytes<double>(nblk);
  s += carve_bytes<double>(3 * ncell);
  s += carve_bytes<unsigned long long>(ncell);
  return s;
}

int validate(extrass_handle h, const extrass_batched* p) {
  if (!p || p->n_cells < 0) return fail(h, EXTRASS_EINVAL, "extrass_batched: bad problem");
  if (p->n_cells == 0) return EXTRASS_OK;
  if (!p->level_count || !p->level_count_d || !p->T_e || !p->n_e || !p->gamma_ion ||
      !p->gamma_pe_table)
    return fail(h, EXTRASS_EINVAL, "extrass_batched: null array");
  if (p->n_gamma_pe < 1)
    return fail(h, EXTRASS_EINVAL, "extrass_batched: empty photoexcitation table");
  for (int64_t c = 0; c < p->n_cells; ++c) {
    const int32_t* Lc = p->level_count + 3 * c;
    for (int z = 0; z < 3; ++z)
      if (Lc[z] < 0 || Lc[z] > kMaxLevels)
        return fail(h, EXTRASS_EINVAL, "extrass_batched: level count outside 0..1023");
    if (Lc[0] < 1 || (Lc[1] == 0 && Lc[2] > 0))
      return fail(h, EXTRASS_EINVAL, "extrass_batched: stage 0 empty or a gap between stages");
  }
  return EXTRASS_OK;
}

Layout make_layout(extrass_handle h, const extrass_batched* p, const extrass_batched_opts* o) {
  Layout y;
  y.fp32 = o && o->factor_fp32 ? 1 : 0;
  y.panel = o && o->panel ? o->panel : (h->batched_panel[y.fp32] ? h->batched_panel[y.fp32] : 32);
  y.per_cu = o && o->per_cu ? o->per_cu
                            : (h->batched_per_cu[y.fp32] ? h->batched_per_cu[y.fp32] : 2);
  int maxB = 1;
  for (int64_t c = 0; c < p->n_cells; ++c)
    for (int z = 0; z < 3; ++z) maxB = std::max(maxB, block_states(p->level_count + 3 * c, z));
  y.ldct = (int)round32(maxB);
  y.G = (int64_t)h->num_cus * y.per_cu;
  const size_t el = y.fp32 ? sizeof(float) : sizeof(double);
  y.fixed = carve_bytes<Blk>(3 * p->n_cells) + carve_bytes<int32_t>(3 * p->n_cells) +
            carve_bytes<int64_t>(p->n_cells + 1) + (size_t)y.G * kCtRows * y.ldct * el + 256 +
            carve_bytes<unsigned int>(1);
  return y;
}

void make_plan(const extrass_batched* p, const Layout& y, size_t ws_bytes, Plan& P) {
  const int64_t C = p->n_cells;
  P.pop.assign(C + 1, 0);
  P.cell_blk.assign(3 * C, -1);
  for (int64_t c = 0; c < C; ++c) {
    const int32_t* Lc = p->level_count + 3 * c;
    P.pop[c + 1] = P.pop[c] + Lc[0] + Lc[1] + Lc[2];
  }
  const size_t budget = ws_bytes > y.fixed ? ws_bytes - y.fixed : 0;
  int64_t c = 0;
  while (c < C) {
    Chunk ch{c, c, (int64_t)P.blk.size(), 0, 0, 0};
    std::vector<Blk> bl;
    while (ch.c1 < C) {
      const int32_t* Lc = p->level_count + 3 * ch.c1;
      const int64_t a = ch.a_elems + cell_matrix_elems(Lc), v = ch.v_elems + cell_vector_elems(Lc);
      const int64_t nb = (int64_t)bl.size() + (Lc[0] > 0) + (Lc[1] > 0) + (Lc[2] > 0);
      if (ch.c1 > ch.c0 && arena_bytes(y, a, v, nb, ch.c1 + 1 - ch.c0) > budget) break;
      for (int z = 0; z < 3; ++z) {
        if (Lc[z] == 0) continue;
        const int B = block_states(Lc, z);
        P.maxB = std::max(P.maxB, B);
        Blk b;
        b.a = ch.a_elems;
        b.v = ch.v_elems;
        b.cell = (int32_t)(ch.c1 - ch.c0);
        b.z = z;
        b.B = B;
        b.L = Lc[z];
        ch.a_elems += round32((int64_t)B * B);
        ch.v_elems += round32(B);
        bl.push_back(b);
      }
      ++ch.c1;
    }
    std::stable_sort(bl.begin(), bl.end(), [](const Blk& u, const Blk& v) { return u.B > v.B; });
    for (size_t i = 0; i < bl.size(); ++i)
      P.cell_blk[3 * (ch.c0 + bl[i].cell) + bl[i].z] = (int32_t)i;
    ch.nblk = (int64_t)bl.size();
    P.blk.insert(P.blk.end(), bl.begin(), bl.end());
    P.chunks.push_back(ch);
    c = ch.c1;
  }
}

size_t min_bytes_of(const extrass_batched* p, const Layout& y) {
  size_t m = 0;
  for (int64_t c = 0; c < p->n_cells; ++c) {
    const int32_t* Lc = p->level_count + 3 * c;
    m = std::max(m, arena_bytes(y, cell_matrix_elems(Lc), cell_vector_elems(Lc), 3, 1));
  }
  return y.fixed + m;
}

size_t all_bytes_of(const extrass_batched* p, const Layout& y) {
  int64_t a = 0, v = 0;
  for (int64_t c = 0; c < p->n_cells; ++c) {
    a += cell_matrix_elems(p->level_count + 3 * c);
    v += cell_vector_elems(p->level_count + 3 * c);
  }
  return y.fixed + arena_bytes(y, a, v, 3 * p->n_cells, p->n_cells);
}

template <class T>
void launch_factor(int panel, dim3 grid, hipStream_t s, const Args& a) {
  switch (panel) {
    case 16: k_factor<T, 16><<<grid, kThreads, 0, s>>>(a); break;
    case 64: k_factor<T, 64><<<grid, kThreads, 0, s>>>(a); break;
    default: k_factor<T, 32><<<grid, kThreads, 0, s>>>(a); break;
  }
}

template <class T>
void launch_backsub(int panel, int nblk, hipStream_t s, const Args& a, int rhs) {
  switch (panel) {
    case 16: k_backsub<T, 16><<<nblk, kThreads, 0, s>>>(a, rhs); break;
    case 64: k_backsub<T, 64><<<nblk, kThreads, 0, s>>>(a, rhs); break;
    default: k_backsub<T, 32><<<nblk, kThreads, 0, s>>>(a, rhs); break;
  }
}

template <class T>
void launch_forward(int panel, int nblk, hipStream_t s, const Args& a) {
  switch (panel) {
    case 16: k_forward<T, 16><<<nblk, kThreads, 0, s>>>(a); break;
    case 64: k_forward<T, 64><<<nblk, kThreads, 0, s>>>(a); break;
    default: k_forward<T, 32><<<nblk, kThreads, 0, s>>>(a); break;
  }
}

// Device tables for all cells, then per-chunk arenas carved from the rest.
struct Carved {
  Blk* blk;
  int32_t* cell_blk;
  int64_t* pop;
  void* ct;
  unsigned int* queue;
  char* arena_base;
  size_t arena_cap;
};

int upload_tables(extrass_handle h, const Plan& P, const Layout& y, void* ws, size_t ws_bytes,
                  hipStream_t s, Carved& cv, int64_t C) {
  Carver cw(ws, ws_bytes);
  cv.blk = cw.take<Blk>(3 * C);
  cv.cell_blk = cw.take<int32_t>(3 * C);
  cv.pop = cw.take<int64_t>(C + 1);
  // column factors of one group of panels per resident work-group
  cv.ct = cw.take<char>((size_t)y.G * kCtRows * y.ldct * (y.fp32 ? sizeof(float) : sizeof(double)));
  cv.queue = cw.take<unsigned int>(1);
  if (!cw.ok()) return fail(h, EXTRASS_ENOSPACE, "extrass_batched: workspace too small");
  const size_t used = (cw.used + 255) & ~size_t(255);
  cv.arena_base = static_cast<char*>(ws) + used;
  cv.arena_cap = ws_bytes > used ? ws_bytes - used : 0;
  EXTRASS_HIP_TRY(h, hipMemcpyAsync(cv.blk, P.blk.data(), sizeof(Blk) * P.blk.size(),
                                    hipMemcpyHostToDevice, s));
  EXTRASS_HIP_TRY(h, hipMemcpyAsync(cv.cell_blk, P.cell_blk.data(), sizeof(int32_t) * P.cell_blk.size(),
                                    hipMemcpyHostToDevice, s));
  EXTRASS_HIP_TRY(h, hipMemcpyAsync(cv.pop, P.pop.data(), sizeof(int64_t) * P.pop.size(),
                                    hipMemcpyHostToDevice, s));
  // the host vectors go out of scope with the caller's plan: wait for the copies
  EXTRASS_HIP_TRY(h, hipStreamSynchronize(s));
  return EXTRASS_OK;
}

Args chunk_args(const extrass_batched* p, const Layout& y, const Plan& P, const Chunk& ch,
                const Carved& cv, double* pops, int32_t* status) {
  Args a{};
  a.blk = cv.blk + ch.blk0;
  a.nblk = (int)ch.nblk;
  a.ncell = (int)(ch.c1 - ch.c0);
  a.c0 = ch.c0;
  a.seed = p->seed;
  a.L = p->level_count_d;
  a.pop = cv.pop;
  a.T_e = p->T_e;
  a.n_e = p->n_e;
  a.gion = p->gamma_ion;
  a.gpe_tab = p->gamma_pe_table;
  a.n_gpe = p->n_gamma_pe;
  a.alpha0_0 = p->alpha0[0];
  a.alpha0_1 = p->alpha0[1];
  Carver cw(cv.arena_base, cv.arena_cap);
  a.A64 = cw.take<double>(ch.a_elems);
  a.A32 = y.fp32 ? cw.take<float>(ch.a_elems) : nullptr;
  a.S = cw.take<double>(ch.v_elems);
  a.rowsum = y.fp32 ? cw.take<double>(ch.v_elems) : nullptr;
  a.bvec = y.fp32 ? cw.take<double>(ch.v_elems) : nullptr;
  a.scale = y.fp32 ? cw.take<double>(ch.nblk) : nullptr;
  a.red = cw.take<double>(2 * ch.nblk);
  a.rb = cw.take<double>(2 * ch.nblk);
  a.cell_blk = cv.cell_blk + 3 * ch.c0;
  a.gval = cw.take<double>(3 * (ch.c1 - ch.c0));
  a.maxrel = cw.take<unsigned long long>(ch.c1 - ch.c0);
  a.ct = cv.ct;
  a.maxB = P.maxB;
  a.ldct = y.ldct;
  a.queue = cv.queue;
  a.pops = pops;
  a.status = status;
  return a;
}

int run_chunk(extrass_handle h, const Layout& y, const Args& a, int refine, double tol,
              hipStream_t s, hipEvent_t f0 = nullptr, hipEvent_t f1 = nullptr) {
  const int nblk = a.nblk, ncell = a.ncell;
  k_assemble<<<nblk, kThreads, assemble_lds(a), s>>>(a, y.fp32);
  k_zero_queue<<<1, 1, 0, s>>>(a.queue);
  const dim3 grid((unsigned)std::min<int64_t>(y.G, nblk));
  if (f0) EXTRASS_HIP_TRY(h, hipEventRecord(f0, s));
  if (y.fp32)
    launch_factor<float>(y.panel, grid, s, a);
  else
    launch_factor<double>(y.panel, grid, s, a);
  if (f1) EXTRASS_HIP_TRY(h, hipEventRecord(f1, s));
  const int cgrid = (ncell + 255) / 256;
  k_chain<<<cgrid, 256, 0, s>>>(a, 0);
  if (y.fp32)
    launch_backsub<float>(y.panel, nblk, s, a, 0);
  else
    launch_backsub<double>(y.panel, nblk, s, a, 0);
  for (int it = 0; y.fp32 && it < refine; ++it) {
    k_fill_u64<<<(ncell + 255) / 256, 256, 0, s>>>(a.maxrel, ncell);
    k_residual<<<nblk, kThreads, 0, s>>>(a);
    launch_forward<float>(y.panel, nblk, s, a);
    k_chain<<<cgrid, 256, 0, s>>>(a, 1);
    launch_backsub<float>(y.panel, nblk, s, a, 1);
  }
  k_normalise<<<(ncell + 3) / 4, kThreads, 0, s>>>(a, y.fp32 && refine > 0, tol);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}

}  // namespace
}  // namespace extrass

using namespace extrass;

extern "C" int extrass_batched_workspace(extrass_handle h, const extrass_batched* p,
                                         const extrass_batched_opts* o, size_t* min_bytes,
                                         size_t* all_bytes) {
  if (!h || !min_bytes || !all_bytes) return EXTRASS_EINVAL;
  const int v = validate(h, p);
  if (v) return v;
  if (p->n_cells == 0) {
    *min_bytes = *all_bytes = 0;
    return EXTRASS_OK;
  }
  const Layout y = make_layout(h, p, o);
  if (y.panel != 16 && y.panel != 32 && y.panel != 64)
    return fail(h, EXTRASS_EINVAL, "extrass_batched: panel must be 16, 32 or 64");
  if (y.per_cu < 1 || y.per_cu > 8) return fail(h, EXTRASS_EINVAL, "extrass_batched: per_cu 1..8");
  *min_bytes = min_bytes_of(p, y);
  *all_bytes = all_bytes_of(p, y);
  return EXTRASS_OK;
}

extern "C" int extrass_batched_solve(extrass_handle h, const extrass_batched* p,
                                     const extrass_batched_opts* o, double* pops, int32_t* status,
                                     void* ws, size_t ws_bytes, void* stream_) {
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  if (!h) return EXTRASS_EINVAL;
  const int v = validate(h, p);
  if (v) return v;
  if (p->n_cells == 0) return EXTRASS_OK;
  if (!pops || !status || !ws) return fail(h, EXTRASS_EINVAL, "extrass_batched_solve: null pointer");
  const Layout y = make_layout(h, p, o);
  if (y.panel != 16 && y.panel != 32 && y.panel != 64)
    return fail(h, EXTRASS_EINVAL, "extrass_batched: panel must be 16, 32 or 64");
  if (y.per_cu < 1 || y.per_cu > 8) return fail(h, EXTRASS_EINVAL, "extrass_batched: per_cu 1..8");
  if (ws_bytes < min_bytes_of(p, y))
    return fail(h, EXTRASS_ENOSPACE, "extrass_batched_solve: workspace below the minimum");
  const int refine = o ? std::max(0, (int)o->refine) : 0;
  const double tol = o && o->tol > 0.0 ? o->tol : 1e-12;
  Plan P;
  make_plan(p, y, ws_bytes, P);
  Carved cv;
  int r = upload_tables(h, P, y, ws, ws_bytes, stream, cv, p->n_cells);
  if (r) return r;
  for (const Chunk& ch : P.chunks) {
    const Args a = chunk_args(p, y, P, ch, cv, pops, status);
    r = run_chunk(h, y, a, refine, tol, stream);
    if (r) return r;
  }
  return EXTRASS_OK;
}

extern "C" int extrass_batched_tune(extrass_handle h, const extrass_batched* p,
                                    const extrass_batched_opts* o, void* ws, size_t ws_bytes,
                                    void* stream_, int32_t* choice, float* times) {
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  if (!h) return EXTRASS_EINVAL;
  const int v = validate(h, p);
  if (v) return v;
  if (p->n_cells == 0 || !ws) return fail(h, EXTRASS_EINVAL, "extrass_batched_tune: nothing to tune on");
  extrass_batched_opts base{};
  if (o) base = *o;
  const int fp32 = base.factor_fp32 ? 1 : 0;
  const int panels[3] = {16, 32, 64}, per_cus[3] = {1, 2, 4};
  // plan once with the largest candidate so that every candidate runs on the same cells
  extrass_batched_opts big = base;
  big.panel = 64;
  big.per_cu = 4;
  const Layout yb = make_layout(h, p, &big);
  if (ws_bytes < min_bytes_of(p, yb))
    return fail(h, EXTRASS_ENOSPACE, "extrass_batched_tune: workspace below the minimum");
  Plan P;
  make_plan(p, yb, ws_bytes, P);
  const Chunk ch = P.chunks[0];
  Carved cv;
  int r = upload_tables(h, P, yb, ws, ws_bytes, stream, cv, p->n_cells);
  if (r) return r;
  // scratch outputs for the tuning runs: the chunk's populations in the arena's tail
  Args a0 = chunk_args(p, yb, P, ch, cv, nullptr, nullptr);
  hipEvent_t e0, e1;
  EXTRASS_HIP_TRY(h, hipEventCreate(&e0));
  EXTRASS_HIP_TRY(h, hipEventCreate(&e1));
  float best = INFINITY;
  int bp = 32, bc = 2;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Layout y = yb;
      y.panel = panels[i];
      y.per_cu = per_cus[j];
      y.G = (int64_t)h->num_cus * y.per_cu;
      y.fp32 = fp32;
      Args a = a0;
      const int nblk = a.nblk;
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {  // first run warms up
        k_assemble<<<nblk, kThreads, assemble_lds(a), stream>>>(a, fp32);
        k_zero_queue<<<1, 1, 0, stream>>>(a.queue);
        const dim3 grid((unsigned)std::min<int64_t>(y.G, nblk));
        EXTRASS_HIP_TRY(h, hipEventRecord(e0, stream));
        if (fp32)
          launch_factor<float>(y.panel, grid, stream, a);
        else
          launch_factor<double>(y.panel, grid, stream, a);
        EXTRASS_HIP_TRY(h, hipEventRecord(e1, stream));
        EXTRASS_HIP_TRY(h, hipEventSynchronize(e1));
        EXTRASS_HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
      }
      if (times) times[3 * i + j] = ms;
      if (ms < best) {
        best = ms;
        bp = panels[i];
        bc = per_cus[j];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->batched_panel[fp32] = bp;
  h->batched_per_cu[fp32] = bc;
  if (choice) {
    choice[0] = bp;
    choice[1] = bc;
  }
  return EXTRASS_OK;
}
