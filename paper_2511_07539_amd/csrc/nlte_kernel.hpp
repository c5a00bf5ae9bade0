// NLTE statistical equilibrium per (cell, species) (Sec. 2.2; Eqs. A1-A2).
//
// One wavefront solves one (cell, species) system at a time: lane i owns
// level i (up to 64 levels), the rate or flux matrix lives in LDS (row
// stride padded to an odd number of doubles), and wavefronts take work items
// from a global counter until all cells are done.
//
// Per system:
//  1. cold start (Boltzmann within each ion stage, stage ratios from a
//     ground-only ionisation balance) or the caller's guess;
//  2. fixed-point steps n <- n_tot * stationary(R(n)), under-relaxed in
//     log(n) when the change fails to shrink, until max |d ln n| < 0.7 (1.0
//     from a caller's guess); the trust-region Newton below takes over from
//     there; the
//     stationary vector comes from state reduction with pivots formed as sums
//     of off-diagonal rates (Grassmann-Taksar-Heyman), which involves no
//     subtraction and keeps every component accurate. The matrix is assembled
//     in LDS (one transition per lane at a time) and reduced in registers,
//     one row per lane;
//  3. Newton steps in log(n): the Jacobian scaled by diag(n) is a transposed
//     generator (non-negative off-diagonals, zero column sums), so the Newton
//     system is reduced the same way, the most populated level last, and
//     conservation fixes the free multiple of the null vector. The right-hand
//     side -F is formed as Q(n)^T (P(n) - n), P(n) the fixed-point map above:
//     the same vector as the net inflow, without the cancellation of gross
//     inflow against outflow that would limit accuracy to ~1e-9 in weakly
//     coupled ion stages. A trust radius on max |d ln n| and a decrease test
//     on sum (P(n)/n - 1)^2 globalise the iteration.
// Convergence: max |d ln n| < tol with max |P(n)/n - 1| < tol; or, after a
// full Newton step s, a predicted next step below tol / 10 with the residual
// below tol (the step after s is predicted as (s / s'^2) s^2 when a full step
// s' preceded s, else as s scaled by the residual's reduction); or, with the
// residual below tol, a step below 1e-11 that has stopped shrinking (for tol
// under that floor). Every exit counted as converged has met the residual
// test.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "atom.hpp"
#include "common.hpp"

namespace extrass {

struct NArgs {
  int S, N, T;
  int64_t C;
  double t_exp;
  const int32_t* off;
  const int32_t* toff;
  const int32_t* nstage;
  const int32_t* lv_ion;
  const int32_t* lv_gnext;
  const double* lv_E;
  const double* lv_g;
  const double* lv_share;
  const double* t_pack;   // [T*6] A lambda^3/(8 pi), A, g_u/g_l, g_l/g_u, 8.629e-6 Upsilon/g_u, dE
  const int32_t* t_idx;   // [T*4] lower, upper (species-local), global index, 0
  const double* alpha0;
  const double* T_e;
  const double* n_e;
  const double* n_species;
  const double* gamma_ion;
  const double* gamma_pe;
  const double* gamma_pi;  // [C*N] photoionisation per level, or NULL
  int max_iter;
  double tol;
  int use_guess;
  int warm_budget;
  double* pops;
  int32_t* status;
  int32_t* iters;
  unsigned long long* queue;
  int NP;   // LDS row stride in doubles (whole-system layout)
  int gsz;  // doubles of LDS holding G (whole-system layout)
  int block_rows;  // lanes of the stage blocks of the largest species, rounded up to even
};

// Kernel launchers, one translation unit each (compiled in parallel):
// stage-block kernels for blocks of at most ntb states (FP64, or with the
// fixed-point steps reduced in FP32), whole-system kernels for species of at
// most nt levels. Return false for an unsupported size.
bool launch_nlte_blocks(int ntb, unsigned blocks, size_t lds, hipStream_t st, const NArgs& A);
bool launch_nlte_blocks_mixed(int ntb, unsigned blocks, size_t lds, hipStream_t st, const NArgs& A);
bool launch_nlte_whole(int nt, unsigned blocks, size_t lds, hipStream_t st, const NArgs& A);

namespace {

constexpr double kBoltzmann = 1.380649e-16;  // erg/K
// A warm guess whose first fixed-point step changes no population by more
// than this factor in log n goes straight to Newton.
constexpr double kNearRoot = 1e-2;

// Everything one system needs, held per wave (uniform values) or per lane.
struct Sys {
  int64_t c;
  int s, base, Ns, t0, t1, nst;
  double T, ne, kT, ikT, isqT, ntot;
  double gion[3], rec[3];
  // lane-owned level data
  int z, gnext;
  double E, g, share;
  // row table in LDS: row i of G starts at rt[i].x and holds columns
  // rt[i].y, rt[i].y + 1, ... (element (i, j) at rt[i].x + j - rt[i].y)
  const int2* rt;
};

__device__ __forceinline__ double beta_sobolev(double tau) {
  return tau <= 0.0 ? 1.0 : -expm1(-tau) / tau;
}

__device__ __forceinline__ double dbeta_sobolev(double tau) {
  if (tau <= 0.0) return 0.0;
  if (tau < 1e-3) return -0.5 + tau * (1.0 / 3.0 - tau * (1.0 / 8.0 - tau / 30.0));
  return (exp(-tau) * (1.0 + tau) - 1.0) / (tau * tau);
}

// Fills G[i][j] (i != j) with rs_i * R_ij at populations n (lane i holds n_i),
// rs_i = n_i when rowscale (fluxes) else 1 (rates). With hb (the relative
// fixed-point residual h_j = P(n)_j / n_j - 1 of every level, in LDS), lane i
// gets the Newton right-hand side -F_i = (Q^T H)_i = sum_j h_j G_ji -
// h_i sum_j G_ij (flux form): the same vector as inflow - outflow with its
// sign flipped, but formed from the small h, so without the cancellation of
// gross inflow against outflow. With jac, the derivative of the radiative
// fluxes through beta_S(tau(n)) is then added, which turns G into the
// diag(n)-scaled Newton matrix.
//
// Row i and column i of the matrix can be nonzero only for levels in
// [rlo, rhi] (lane i's own range: its ion stage and the next stage's ground,
// and for a ground state also the stage below it); only that range is
// cleared and summed.
__device__ __forceinline__ int gat(const int2* rt, int i, int j) {
  const int2 r = rt[i];
  return r.x + j - r.y;
}

__device__ __forceinline__ void assemble(const NArgs& A, const Sys& y, double* G, double* nb, double n_mine,
                         bool rowscale, const double* hb, double h_mine, bool jac, double& rhs,
                         int rlo, int rhi) {
  const int lane = threadIdx.x;
  const int Ns = y.Ns;
  const int2* rt = y.rt;
  double* myrow = G + (lane < Ns ? rt[lane].x - rlo : 0);  // element (lane, j) at myrow[j]
  if (lane < Ns) {
    nb[lane] = n_mine;
    for (int j = rlo; j <= rhi; ++j) myrow[j] = 0.0;
  }
  __syncthreads();
  const double* gpe = A.gamma_pe ? A.gamma_pe + y.c * A.T : nullptr;
#pragma unroll 4
  for (int t = y.t0 + lane; t < y.t1; t += 64) {
    const int4 ix = reinterpret_cast<const int4*>(A.t_idx)[t];
    const int l = ix.x, u = ix.y;
    const double2 p01 = reinterpret_cast<const double2*>(A.t_pack)[3 * t];
    const double2 p23 = reinterpret_cast<const double2*>(A.t_pack)[3 * t + 1];
    const double2 p45 = reinterpret_cast<const double2*>(A.t_pack)[3 * t + 2];
    const double Ad = p01.y, gul = p23.x, glu = p23.y;
    const double qul = p45.x * y.isqT;
    const double qlu = qul * gul * exp(-p45.y * y.ikT);
    const double nl = nb[l], nu = nb[u];
    const double tau = (p01.x * A.t_exp) * (gul * nl - nu);
    const double p = gpe ? gpe[ix.z] : 0.0;
    const double down = Ad * beta_sobolev(tau) + y.ne * qul + glu * p;
    const double up = y.ne * qlu + p;
    G[gat(rt, u, l)] = (rowscale ? nu : 1.0) * down;
    G[gat(rt, l, u)] = (rowscale ? nl : 1.0) * up;
  }
  if (lane < Ns && y.gnext >= 0) {
    const double rs = rowscale ? n_mine : 1.0;
    const double rsg = rowscale ? nb[y.gnext] : 1.0;
    // the stage's ionisation rate plus the level's photoionisation rate
    const double gpi = A.gamma_pi ? A.gamma_pi[y.c * A.N + y.base + lane] : 0.0;
    myrow[y.gnext] += rs * (y.gion[y.z] + gpi);
    G[gat(rt, y.gnext, lane)] += rsg * y.rec[y.z] * y.share;
  }
  __syncthreads();
  if (hb) {
    // -F_i = (Q^T H)_i = sum_j h_j G_ji - h_i sum_j G_ij with H = P(n) - n
    double in = 0.0, out = 0.0;
    if (lane < Ns) {
      for (int j = rlo; j <= rhi; ++j) {
        out += myrow[j];
        in += hb[j] * G[gat(rt, j, lane)];
      }
    }
    rhs = in - h_mine * out;
  }
  if (jac) {
    __syncthreads();
#pragma unroll 4
    for (int t = y.t0 + lane; t < y.t1; t += 64) {
      const int4 ix = reinterpret_cast<const int4*>(A.t_idx)[t];
      const int l = ix.x, u = ix.y;
      const double2 p01 = reinterpret_cast<const double2*>(A.t_pack)[3 * t];
      const double gul = A.t_pack[6 * t + 2];
      const double Ad = p01.y;
      const double nl = nb[l], nu = nb[u];
      const double K = p01.x * A.t_exp;
      const double tau = K * (gul * nl - nu);
      const double db = dbeta_sobolev(tau);
      if (db != 0.0) {
        const double du = -nu * Ad * db * K;
        const double dl = nu * Ad * db * K * gul;
        G[gat(rt, u, l)] += du * nu;
        G[gat(rt, l, u)] += -dl * nl;
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int perm(int a, int big, int last) {
  return a == big ? last : (a == last ? big : a);
}

__device__ __forceinline__ float read_lane(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

__device__ __forceinline__ double read_lane(double v, int k) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, k);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), k);
  return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

// State reduction of the generator in G (off-diagonal entries, row i -> j),
// visiting states in the order perm(0..Ns-1) (the level `big` swapped to the
// end). Solves x^T G = b^T with x_last = 0 when rhs, and the homogeneous
// problem with pi_last = 1. Lane a holds b, x and pi of permuted position a.
// Returns false when a pivot is not positive (reducible chain).
//
// Each lane copies its row into registers (NT >= Ns, a compile-time size);
// the reduction then runs unrolled on registers: at step k every lane sums its
// remaining row entries and lane k's sum is the pivot, lane k publishes its
// row through a small LDS buffer, and the other lanes update their rows with
// it. Entries beyond Ns stay zero. The diagonal is never read. Matrix and
// right-hand side are multiplied by `scale` (a power of two) as they are
// loaded, which leaves x and pi unchanged; T = float gives the
// single-precision reduction.
template <int NT, class T>
__device__ __forceinline__ bool reduce_solve(const double* G, int NP, int Ns, int big, bool rhs,
                                             double b_perm_in, double scale, T* rowbuf, double* out) {
  const int lane = threadIdx.x;
  const int last = Ns - 1;
  const bool live = lane < Ns;
  const int my_row = live ? perm(lane, big, last) : 0;
  T g[NT];
#pragma unroll
  for (int b = 0; b < NT; ++b)
    g[b] = (live && b < Ns && b != lane) ? (T)(scale * G[my_row * NP + perm(b, big, last)]) : T(0);
  // the pivot-row buffer overlays G: keep every row load ahead of its stores
  __asm__ volatile("" ::: "memory");
  T b_perm = (T)(scale * b_perm_in);
  T S_mine = T(0);
  bool ok = true;
#pragma unroll
  for (int k = 0; k < NT - 1; ++k) {
    if (k < last) {
      T part = T(0);
#pragma unroll
      for (int b = k + 1; b < NT; ++b) part += g[b];
      const T S = read_lane(part, k);
      if (!(S > T(0))) ok = false;
      if (lane == k) {
        S_mine = S;
#pragma unroll
        for (int b = k + 1; b < NT; ++b) rowbuf[b] = g[b];
      }
      __builtin_amdgcn_wave_barrier();
      const T invS = T(1) / S;
      const T f = g[k] * invS;
      // eight columns at a time, so that only eight broadcast values are live
#pragma unroll
      for (int b0 = k + 1; b0 < NT; b0 += 8) {
#pragma unroll
        for (int b = b0; b < b0 + 8 && b < NT; ++b) g[b] += f * rowbuf[b];
        __builtin_amdgcn_sched_barrier(0);
      }
      if (rhs) {
        const T bk = read_lane(b_perm, k);
        if (live && lane > k) b_perm += bk * rowbuf[lane] * invS;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  T x = T(0), pi = lane == last ? T(1) : T(0);
#pragma unroll
  for (int k = NT - 2; k >= 0; --k) {
    if (k < last) {
      const T gk = (live && lane > k) ? g[k] : T(0);
      const T sx = rhs ? wave_sum(x * gk) : T(0);
      const T sp = wave_sum(pi * gk);
      const T Sk = read_lane(S_mine, k);
      const T bk = rhs ? read_lane(b_perm, k) : T(0);
      if (lane == k) {
        x = (sx - bk) / Sk;
        pi = sp / Sk;
      }
    }
  }
  out[0] = (double)x;
  out[1] = (double)pi;
  return ok;
}


// ---- stage-block reduction ---------------------------------------------------
// A level exchanges population only with the levels of its own ion stage and
// with the next stage's ground state (ionisation into it, recombination out of
// it). Block z holds [the excited levels of stage z][the ground of z][the
// ground of z+1, below the top stage]; the ground rows appear in two blocks,
// each copy holding the columns of its block. Reducing the excited levels of
// every block is the state reduction of the whole system in an order that
// skips only exact zeros. The ground states left form a birth-death chain,
// solved in closed form with the most populated ground as reference, and
// back-substitution gives the excited levels. The blocks sit side by side in
// one wavefront (one block row per lane) and are reduced in lockstep.
// LDS of the stage-block reduction (doubles, in the space of the assembled
// matrix): pivot rows and the ground-pair values, then the eliminated rows
// [64][NTB + 1] and the published (x, pi) [64][2].
constexpr int kBlockScratch = 114;
// rows: the lanes the stage blocks take, rounded up to even (keeps pv 16-byte
// aligned): eliminated rows [rows][ntb + 1], then (x, pi) [rows][2]
constexpr int block_scratch(int ntb, int rows) { return kBlockScratch + rows * (ntb + 3); }

struct Blocks {
  int nst;
  int st[4];    // first level (the ground) of each stage; st[z] = Ns for z >= nst
  int nex[3];   // excited levels of each stage
  int B[3];     // states of each block
  int base[4];  // first lane of each block
};

__device__ __forceinline__ Blocks make_blocks(const Sys& y) {
  Blocks k;
  k.nst = y.nst;
  const bool live = (int)threadIdx.x < y.Ns;
#pragma unroll
  for (int z = 0; z < 3; ++z) {
    const uint64_t m = __ballot(live && y.z == z);
    k.st[z] = (z < y.nst && m) ? (int)__ffsll((unsigned long long)m) - 1 : y.Ns;
  }
  k.st[3] = y.Ns;
  k.base[0] = 0;
#pragma unroll
  for (int z = 0; z < 3; ++z) {
    const bool has = z < k.nst;
    k.nex[z] = has ? k.st[z + 1] - k.st[z] - 1 : 0;
    k.B[z] = has ? k.nex[z] + 1 + (z + 1 < k.nst ? 1 : 0) : 0;
    k.base[z + 1] = k.base[z] + k.B[z];
  }
  return k;
}

// An int every lane holds, read into a scalar register.
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

// 1/S for a positive normal S: the hardware reciprocal refined by two Newton
// steps (error within a few ulps), without the scaling a full division does
// for operands near the ends of the exponent range.
__device__ __forceinline__ double rcp_pos(double S) {
  double r = __builtin_amdgcn_rcp(S);
  double e = fma(-S, r, 1.0);
  r = fma(r, e, r);
  e = fma(-S, r, 1.0);
  return fma(r, e, r);
}
// The single-precision counterpart: one Newton step on the hardware estimate.
__device__ __forceinline__ float rcp_pos(float S) {
  const float r = __builtin_amdgcn_rcpf(S);
  return fmaf(r, fmaf(-S, r, 1.0f), r);
}

// A pivot the reduction can divide by: positive, and in FP32 also normal
// (the reciprocal of a subnormal overflows).
__device__ __forceinline__ bool pivot_ok(double S) { return S > 0.0; }
__device__ __forceinline__ bool pivot_ok(float S) { return S >= 1.17549435e-38f && S <= 3.4e38f; }

// Solves x^T Q = b^T (rhs, with x of the ground `pin` fixed at 0) and the
// stationary problem (pi of the ground `pin` = 1) for the generator whose
// off-diagonal entries are in G. b_nat: lane = level. Lane l < Ns receives
// (x_l, pi_l) in out. LDS: scratch >= block_scratch(NTB, nrow) doubles
// (16-byte aligned), xo/po >= 64 doubles each; nrow >= the lanes of the blocks.
// Returns false when a pivot is not positive.
//
// T = float reduces in single precision: rows, pivots, elimination and
// back-substitution; the ground chain stays in FP64. Meant for the
// stationary problem, whose reduction adds and multiplies positive numbers
// only, so every component keeps FP32's relative accuracy. The matrix and
// the right-hand side are first scaled by one power of two that takes the
// largest entry of the system into [1, 2) (x and pi are unchanged by a
// common scale), and pi of the reference ground is 2^100 instead of 1: rates
// down to ~1e-38 of the largest and populations down to ~1e-68 of the
// reference stay normal, and the products pi_j a_jr of the back-substitution
// stay below ~2^107. A pivot or a pi outside the normal FP32 range returns
// false.
template <int NTB, class T = double>
__device__ __forceinline__ bool reduce_blocks(const double* G, const int2* rt, int Ns, int nrow,
                                              const Blocks& k,
                                              bool rhs, double b_nat, int pin, double* scratch,
                                              double* xo, double* po, double* out) {
  static_assert(NTB <= 32, "row slots 32 and 33 carry the pivot and right-hand side");
  constexpr bool kSingle = sizeof(T) == 4;
  using T2 = typename std::conditional<kSingle, float2, double2>::type;
  const int lane = threadIdx.x;
  // [3][34]: pivot rows with the pivot and right-hand side in slots 32, 33
  T* rows = reinterpret_cast<T*>(scratch);
  double* small = scratch + 102;  // reduced rates and right-hand sides of the ground pairs
  // The lane's block quantities are selected by its block z among values
  // every lane holds. Selecting among the descriptor's array elements
  // directly made the compiler index a stack copy of the descriptor (a
  // scratch load per use); read as scalars first, they are register selects.
  const int base1 = rfl(k.base[1]), base2 = rfl(k.base[2]);
  const int z = lane < base1 ? 0 : (lane < base2 ? 1 : 2);
  const bool live = z < k.nst && lane < rfl(k.base[3]);
  const int base = z == 0 ? rfl(k.base[0]) : (z == 1 ? base1 : base2);
  const int r = lane - base;
  const int nex = live ? (z == 0 ? rfl(k.nex[0]) : (z == 1 ? rfl(k.nex[1]) : rfl(k.nex[2]))) : 0;
  const int B = live ? (z == 0 ? rfl(k.B[0]) : (z == 1 ? rfl(k.B[1]) : rfl(k.B[2]))) : 0;
  // the lane's block bounds and row-table entry, once for the unrolled loop
  const int st0 = rfl(k.st[0]), st1 = rfl(k.st[1]), st2 = rfl(k.st[2]), st3 = rfl(k.st[3]);
  const int st_z = z == 0 ? st0 : (z == 1 ? st1 : st2);
  const int sn_z = z == 0 ? st1 : (z == 1 ? st2 : st3);
  const int my_lev = live ? (r < nex ? st_z + 1 + r : (r == nex ? st_z : sn_z)) : 0;
  const int2 my_rt = rt[my_lev];
  double sc = 1.0;  // the common power-of-two scale (FP32 only)
  if constexpr (kSingle) {
    double m = 0.0;
#pragma unroll
    for (int b = 0; b < NTB; ++b) {
      const int lev_b = b < nex ? st_z + 1 + b : (b == nex ? st_z : sn_z);
      m = fmax(m, (live && b < B && b != r) ? fabs(G[my_rt.x + lev_b - my_rt.y]) : 0.0);
    }
    m = wave_max(m);
    const int e = m > 0.0 ? -ilogb(m) : 0;
    sc = uniform_d(ldexp(1.0, e < 1000 ? e : 1000));
  }
  T g[NTB];
#pragma unroll
  for (int b = 0; b < NTB; ++b) {
    const int lev_b = b < nex ? st_z + 1 + b : (b == nex ? st_z : sn_z);
    g[b] = (live && b < B && b != r) ? (T)(sc * G[my_rt.x + lev_b - my_rt.y]) : T(0);
  }
  // the scratch below overlays G: keep every row load ahead of its stores
  __asm__ volatile("" ::: "memory");
  // right-hand side: a ground's entry is counted in its own block only
  double bbd = __shfl(b_nat, my_lev, 64);
  T bb = (rhs && live && r <= nex) ? (T)(sc * bbd) : T(0);
  T* myrow = rows + 34 * z;
  bool ok = true;
  T my_inv = T(0);  // 1 / pivot of this lane's state, kept for the back-substitution
  // a block has at most NTB - 1 excited levels (the top stage has no next ground)
#pragma unroll
  for (int kk = 0; kk < NTB - 1; ++kk) {
    // row sum over the remaining states in 8 partial sums (the first term of
    // each seeds it: no additions of zero)
    T acc[8];
#pragma unroll
    for (int b = kk + 1; b < NTB; ++b) {
      const int a = (b - kk - 1) & 7;
      acc[a] = b - kk - 1 < 8 ? g[b] : acc[a] + g[b];
    }
    const int nrem = NTB - kk - 1;
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (a >= nrem) acc[a] = T(0);
    const T part = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    const bool act = live && kk < nex;
    // the pivot lane of each block publishes its row, its row sum (the pivot)
    // and its right-hand side
    if (act && r == kk) {
#pragma unroll
      for (int b = kk + 1; b < NTB; ++b) myrow[b] = g[b];
      myrow[32] = part;
      myrow[33] = bb;
    }
    __builtin_amdgcn_wave_barrier();
    if (act) {
      const T S = myrow[32], bk = myrow[33];
      if (!pivot_ok(S)) ok = false;
      const T inv = rcp_pos(S);
      if (r == kk) my_inv = inv;
      const T f = g[kk] * inv;
#pragma unroll
      // in chunks of 8: the chunk's pivot-row reads are issued together, then
      // its updates (left to itself, the scheduler kept the register
      // pressure down by waiting on each read before the next; 16 or 24 per
      // chunk spill more and are slower)
      for (int b0 = kk + 1; b0 < NTB; b0 += 8) {
        T p[8];
#pragma unroll
        for (int b = b0; b < b0 + 8 && b < NTB; ++b) p[b - b0] = myrow[b];
        __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);   // LDS reads
        __builtin_amdgcn_sched_group_barrier(0x002, 16, 0);  // then vector ALU
#pragma unroll
        for (int b = b0; b < b0 + 8 && b < NTB; ++b) g[b] += f * p[b - b0];
        __builtin_amdgcn_sched_barrier(0);
      }
      // every lane reads (no branch around the load); only r > kk keeps it
      const T mr = myrow[r < NTB ? r : NTB - 1];
      bb += (rhs && r > kk) ? bk * mr * inv : T(0);
    }
    __builtin_amdgcn_wave_barrier();
  }
  // reduced rates between the ground pair of each block: u_z (g_z -> g_z+1)
  // in the own-ground row, d_z (g_z+1 -> g_z) in the next-ground row
  T cu = T(0), cd = T(0);
#pragma unroll
  for (int b = 0; b < NTB; ++b) {
    cu = (b == nex + 1) ? g[b] : cu;
    cd = (b == nex) ? g[b] : cd;
  }
  if (live && r == nex && B == nex + 2) { small[2 * z] = (double)cu; small[6 + 2 * z] = (double)bb; }
  if (live && r == nex && B == nex + 1) small[6 + 2 * z] = (double)bb;
  if (live && r == nex + 1) { small[2 * z + 1] = (double)cd; small[6 + 2 * z + 1] = (double)bb; }
  __builtin_amdgcn_wave_barrier();
  // ground-state chain
  const int K = k.nst;
  double u[2], d[2], bg[3], pg[3], xg[3];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    u[q] = uniform_d(q + 1 < K ? small[2 * q] : 1.0);
    d[q] = uniform_d(q + 1 < K ? small[2 * q + 1] : 1.0);
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    bg[q] = uniform_d((rhs && q < K) ? small[6 + 2 * q] + (q > 0 ? small[6 + 2 * (q - 1) + 1] : 0.0) : 0.0);
    pg[q] = 0.0;
    xg[q] = 0.0;
  }
  pg[pin] = kSingle ? 0x1p100 : 1.0;
#pragma unroll
  for (int q = 1; q < 3; ++q)
    if (q > pin && q < K) pg[q] = pg[q - 1] * u[q - 1] / d[q - 1];
#pragma unroll
  for (int q = 1; q >= 0; --q)
    if (q < pin) pg[q] = pg[q + 1] * d[q] / u[q];
  if (rhs) {
    // reduce the chain towards `pin` from both ends; each pivot is the one
    // remaining rate of its state and carries the right-hand side along
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (q < pin) bg[q + 1] += bg[q];
#pragma unroll
    for (int q = 2; q >= 1; --q)
      if (q > pin && q < K) bg[q - 1] += bg[q];
#pragma unroll
    for (int q = 1; q < 3; ++q)
      if (q > pin && q < K) xg[q] = (xg[q - 1] * u[q - 1] - bg[q]) / d[q - 1];
#pragma unroll
    for (int q = 1; q >= 0; --q)
      if (q < pin) xg[q] = (xg[q + 1] * d[q] - bg[q]) / u[q];
  }
  // back-substitution: every eliminated row goes to LDS once (G is no longer
  // needed); then, state by state in reverse elimination order, the state's
  // (x, pi) is published and the rows c < j of its block add x_j * a[j][c];
  // the ground rows first
  const double xg0 = uniform_d(xg[0]), xg1 = uniform_d(xg[1]), xg2 = uniform_d(xg[2]);
  const double pg0 = uniform_d(pg[0]), pg1 = uniform_d(pg[1]), pg2 = uniform_d(pg[2]);
  const double gz_x = z == 0 ? xg0 : (z == 1 ? xg1 : xg2);
  const double gz_p = z == 0 ? pg0 : (z == 1 ? pg1 : pg2);
  const double gn_x = z == 0 ? xg1 : (z == 1 ? xg2 : 0.0);
  const double gn_p = z == 0 ? pg1 : (z == 1 ? pg2 : 0.0);
  T xm = T(0), pm = T(0);
  if (live && r == nex) { xm = (T)gz_x; pm = (T)gz_p; }
  if (live && r == nex + 1) { xm = (T)gn_x; pm = (T)gn_p; }
  constexpr int LDW = NTB + 1;
  T* Ld = reinterpret_cast<T*>(scratch + kBlockScratch);  // [nrow][LDW] eliminated rows, by lane
  T2* pv = reinterpret_cast<T2*>(Ld + nrow * LDW);          // [nrow] (x, pi) by lane
  if (live) {
#pragma unroll
    for (int b = 0; b < NTB; ++b) Ld[lane * LDW + b] = g[b];
    if (r == nex || r == nex + 1) pv[lane] = T2{xm, pm};
  }
  __builtin_amdgcn_wave_barrier();
  T tx = T(0), tp = T(0);
  if (live && r < nex) {
    const int jg = base + nex;  // own ground, then the next ground
    const T ag = Ld[jg * LDW + r];
    const T2 vg = pv[jg];
    tx += vg.x * ag;
    tp += vg.y * ag;
    if (B > nex + 1) {
      const T an = Ld[(jg + 1) * LDW + r];
      const T2 vn = pv[jg + 1];
      tx += vn.x * an;
      tp += vn.y * an;
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int kk = NTB - 2; kk >= 0; --kk) {
    if (live && r == kk && kk < nex) {
      xm = rhs ? (tx - bb) * my_inv : T(0);
      pm = tp * my_inv;
      pv[lane] = T2{xm, pm};
    }
    __builtin_amdgcn_wave_barrier();
    if (live && r < kk && kk < nex) {
      const int j = base + kk;
      const T a = Ld[j * LDW + r];
      const T2 v = pv[j];
      tx += v.x * a;
      tp += v.y * a;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if constexpr (kSingle)
    if (live && r <= nex && !pivot_ok(pm)) ok = false;
  // back to level order
  if (live && r <= nex) {
    xo[my_lev] = (double)xm;
    po[my_lev] = (double)pm;
  }
  __builtin_amdgcn_wave_barrier();
  out[0] = lane < Ns ? xo[lane] : 0.0;
  out[1] = lane < Ns ? po[lane] : 0.0;
  return __ballot(!ok) == 0ull;
}

// Solves one (cell, species) system; returns the iteration count, or -1.
//
// Written as a loop over phases so that the matrix assembly and the state
// reduction each appear once (both are large once unrolled):
//  FIXED  - one fixed-point step (stationary vector of R(n), relaxed in log n);
//  RESID  - fixed-point residual h = P(n)/n - 1 at the current n;
//  NEWTON - Newton step from the scaled Jacobian with right-hand side Q^T H;
//  TRIAL  - fixed-point residual at a trial point inside the trust radius.
// MIX: the fixed-point steps reduce their stationary problem in FP32 (but
// the first step from a guess, which may serve as the residual at the
// guess); residuals and Newton systems stay FP64, so every exit test is that
// of the FP64 solve. A step whose FP32 pivots or stationary components leave
// the normal range is assembled again and reduced in FP64.
template <int NT, int NTB, bool MIX = false>
__device__ __forceinline__ int solve_system(const NArgs& A, const Sys& y, double* G, double* nb,
                                         double* hb,
                            double* rowbuf, double& n, int max_iter, int check_at, bool warm,
                            int& used) {
  enum { FIXED, RESID, NEWTON, TRIAL };
  const int lane = threadIdx.x;
  const bool live = lane < y.Ns;
  const int last = y.Ns - 1;
  used = 0;
  if (max_iter <= 0) return -1;
  int phase = FIXED, it = 0, bt = 0, best_it = 0;
  double omega = 1.0, prev = INFINITY, Delta = 1.0, best_step = INFINITY, last_full = 0.0;
  Blocks bl{};
  int rlo = 0, rhi = y.Ns - 1;  // the levels row and column `lane` can couple to
  if constexpr (NTB > 0) {
    bl = make_blocks(y);
    if (live) {
      const int st = y.z == 0 ? bl.st[0] : (y.z == 1 ? bl.st[1] : bl.st[2]);
      const int below = y.z == 1 ? bl.st[0] : (y.z == 2 ? bl.st[1] : 0);
      rlo = (lane == st && y.z > 0) ? below : st;
      rhi = y.z + 1 < bl.nst ? (y.z == 0 ? bl.st[1] : bl.st[2]) : y.Ns - 1;
    }
  }
  {
    // row table of G: rows packed back to back, each holding its own range
    // (stage blocks), or the dense layout with stride NP (whole system)
    int off = lane * A.NP;
    if constexpr (NTB > 0) {
      const int w = live ? rhi - rlo + 1 : 0;
      int inc = w;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
      }
      off = inc - w;
    }
    if (live) const_cast<int2*>(y.rt)[lane] = make_int2(off, rlo);
  }
  double h = 0.0, x = 0.0, step = 0.0, taken = 0.0, trial = 0.0, phi = 0.0, res = 0.0;
  bool force64 = false;  // MIX: redo this fixed-point step in FP64
  for (;;) {
    const bool newton = phase == NEWTON;
    const double at = phase == TRIAL ? trial : n;
    if (newton && live) hb[lane] = h;
    double rhs = 0.0, xo[2];
    assemble(A, y, G, nb, at, newton, newton ? hb : nullptr, h, newton, rhs, rlo, rhi);
    int big = last;
    double b_perm = 0.0;
    bool ok = false, done = false;
    if constexpr (NTB > 0) {
      // the most populated ground state is the chain's reference
      int pin = 0;
      double best = -1.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double v = uniform_d(__shfl(n, q < y.nst ? bl.st[q] : 0, 64));
        if (q < y.nst && v > best) {
          best = v;
          pin = q;
        }
      }
      if constexpr (MIX) {
        if (phase == FIXED && !force64 && !(warm && it == 0)) {
          ok = reduce_blocks<NTB, float>(G, y.rt, y.Ns, A.block_rows, bl, false, 0.0, pin, rowbuf, nb, hb, xo);
          if (!ok) {
            force64 = true;
            continue;
          }
        } else {
          ok = reduce_blocks<NTB, double>(G, y.rt, y.Ns, A.block_rows, bl, newton, rhs, pin, rowbuf, nb, hb, xo);
        }
        force64 = false;
      } else {
        ok = reduce_blocks<NTB>(G, y.rt, y.Ns, A.block_rows, bl, newton, rhs, pin, rowbuf, nb, hb, xo);
      }
      done = true;
    } else if (newton) {
      // most populated level (first one on ties) goes last
      const double nmax = wave_max(live ? n : -1.0);
      const uint64_t bm = __ballot(live && n == nmax);
      big = __ffsll((unsigned long long)bm) - 1;
      b_perm = __shfl(rhs, live ? perm(lane, big, last) : 0, 64);
    }
    if constexpr (NTB == 0)
      if (!done) ok = reduce_solve<NT, double>(G, A.NP, y.Ns, big, newton, b_perm, 1.0, rowbuf, xo);
    if (!ok) return -1;
    if (phase == FIXED) {
      const double pp = xo[1];
      const double psum = wave_sum(live ? pp : 0.0);
      const double nw = live ? y.ntot * (pp / psum) : 0.0;
      const double change = wave_max(live ? fabs(log(nw / n)) : 0.0);
      if (warm && it == 0 && change < kNearRoot) {
        // a guess this close to the root (the previous global iteration's
        // solution): this solve is already the residual at the guess, and
        // Newton starts from the guess itself
        h = live ? nw / n - 1.0 : 0.0;
        ++it;
        used = it;
        if (it >= max_iter || (check_at > 0 && it == check_at)) return -1;
        phase = NEWTON;
        continue;
      }
      if (change > 0.999 * prev) omega = uniform_d(omega * 0.5 > 1.0 / 1024 ? omega * 0.5 : 1.0 / 1024);
      prev = change;
      const double v = live ? exp((1.0 - omega) * log(n) + omega * log(nw)) : 0.0;
      const double tot = wave_sum(v);
      n = live ? v * (y.ntot / tot) : 0.0;
      ++it;
      // the fixed-point phase ends at a change below 0.7 from the cold start,
      // 1.0 from a guess checked against a warm budget (a learned guess),
      // 0.1 from a guess trusted without one (the previous global
      // iteration's populations: more fixed-point steps, fewer Newton steps)
      if (change < (warm ? (check_at == 0 ? 0.1 : 1.0) : 0.7) || it >= 60) phase = RESID;
      used = it;
      if (it >= max_iter || (check_at > 0 && it == check_at)) return -1;
      best_it = it;
    } else if (phase == RESID || phase == TRIAL) {
      const double pp = xo[1];
      const double psum = wave_sum(live ? pp : 0.0);
      const double hv = live ? y.ntot * (pp / psum) / at - 1.0 : 0.0;
      if (phase == RESID) {
        h = hv;
        phase = NEWTON;
      } else {
        const double phi2 = wave_sum(hv * hv);
        const double res2 = wave_max(fabs(hv));
        if (phi2 < phi || res2 < 1e-14) {  // accept the trial point
          n = trial;
          h = hv;
          if (taken >= 0.99 * Delta) Delta = uniform_d(2.0 * Delta < 30.0 ? 2.0 * Delta : 30.0);
          ++it;
          used = it;
          if (it >= max_iter) return -1;
          // warm-start check: still far from the root after the budget
          if (check_at > 0 && it == check_at && !(res2 < 1e-6)) return -1;
          // In the quadratic end game the next full Newton step is about
          // (s / s_prev^2) s^2 for this full step s and the one before it,
          // or, after a first full step, (s / r) r_new: the step scaled by
          // the reduction of the residual it was taken from. When that is
          // below tol/10 and the residual is already below tol, the
          // verifying Newton step is skipped.
          if (taken == step) {
            const double pred = last_full > 0.0 ? (step / (last_full * last_full)) * step * step
                                                : step * (res2 / res);
            if (pred < 0.1 * A.tol && res2 < A.tol) return it;
          }
          last_full = taken == step ? step : 0.0;
          phase = NEWTON;
        } else {
          Delta = uniform_d((taken < Delta ? taken : Delta) / 4.0);
          // no trial point lowers the residual: accepted only as a root (the
          // residual test met, the step at rounding level)
          if (++bt >= 40) return (res < A.tol && step < 1e-11) ? it + 1 : -1;
        }
      }
    } else {  // NEWTON
      res = wave_max(fabs(h));
      phi = wave_sum(h * h);
      const int src = live ? perm(lane, big, last) : 0;
      x = __shfl(xo[0], src, 64);
      double pi = __shfl(xo[1], src, 64);
      if (!live) x = pi = 0.0;
      const double sum_n = wave_sum(n), sum_nx = wave_sum(n * x), sum_npi = wave_sum(n * pi);
      const double cst = uniform_d(((y.ntot - sum_n) - sum_nx) / sum_npi);
      x += cst * pi;
      if (!live) x = 0.0;
      step = wave_max(fabs(x));
      if (step < best_step) {
        best_step = step;
        best_it = it;
      }
      // converged; or, with the residual test met, a step at rounding level
      // that has stopped shrinking (tolerances below the step's floor)
      if ((step < A.tol && res < A.tol) || (step < 1e-11 && it - best_it >= 3 && res < A.tol))
        return it + 1;
      bt = 0;
      phase = TRIAL;
    }
    if (phase == TRIAL) {  // trial point in log(n) within the trust radius
      const double scale = uniform_d(step > Delta ? Delta / step : 1.0);
      taken = uniform_d(step * scale);
      const double v = live ? n * exp(scale * x) : 0.0;
      const double tot = wave_sum(v);
      trial = live ? v * (y.ntot / tot) : 0.0;
    }
  }
}

// Cold start: Boltzmann populations within each ion stage at T_e, stage
// ratios from a balance of ionisation against recombination of ground states.
__device__ double cold_start(const Sys& y, bool live) {
  double w = live ? y.g * exp(-y.E / y.kT) : 0.0;
  if (live && w < 1e-250) w = 1e-250;
  double ss[3];
  for (int zz = 0; zz < 3; ++zz) ss[zz] = wave_sum((live && y.z == zz) ? w : 0.0);
  double ratio[3] = {1.0, 1.0, 1.0};
  for (int zz = 1; zz < y.nst; ++zz) {
    const double rc = y.rec[zz - 1];
    double r = rc > 0.0 ? y.gion[zz - 1] / rc : 1e30;
    r = r < 1e-30 ? 1e-30 : (r > 1e30 ? 1e30 : r);
    ratio[zz] = uniform_d(ratio[zz - 1] * r);
  }
  double rsum = 0.0;
  for (int zz = 0; zz < y.nst; ++zz) rsum += ratio[zz];
  rsum = uniform_d(rsum);
  return live ? y.ntot * (ratio[y.z] / rsum) * (w / ss[y.z]) : 0.0;
}

// NTB > 0: stage-block reduction with blocks of at most NTB states (every
// species fits); NTB = 0: whole-system reduction with NT >= the largest species.
template <int NT, int NTB, bool MIX = false>
// Three wavefronts per SIMD (168 VGPRs): the solver is bound by the latency
// of its wave-serial steps, and the third wavefront hides more of it than the
// extra register spills cost.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_nlte(NArgs A) {
  extern __shared__ double smem[];
  double* nb = smem;            // 64 doubles: populations broadcast
  double* hb = smem + 64;       // 64 doubles: fixed-point residuals broadcast
  int2* rt = reinterpret_cast<int2*>(smem + 128);  // 64 entries: the row table of G
  double* G = smem + 192;       // the matrix (row table layout), at least block_scratch(NTB, rows)
  // The stage-block reduction copies its rows out of G into registers before
  // it writes its scratch (pivot rows, pivots), and G is assembled afresh
  // before it is read again, so its scratch shares G's space. The
  // whole-system reduction may redo an FP32 step in FP64 from the same G, so
  // its 64-double pivot-row buffer follows G.
  double* rowbuf = NTB > 0 ? G : G + A.gsz;
  const int lane = threadIdx.x;
  const int64_t items = A.C * A.S;
  for (;;) {
    unsigned long long item = 0;
    if (lane == 0) item = atomicAdd(A.queue, 1ull);
    item = __shfl(item, 0, 64);
    // every lane holds lane 0's value: make it, and what derives from it,
    // scalar
    item = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(item >> 32)) << 32) |
           (unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)item);
    if (item >= (unsigned long long)items) break;
    Sys y;
    y.c = (int64_t)(item / A.S);
    y.s = (int)(item % A.S);
    y.base = __builtin_amdgcn_readfirstlane(A.off[y.s]);
    y.Ns = __builtin_amdgcn_readfirstlane(A.off[y.s + 1]) - y.base;
    y.t0 = __builtin_amdgcn_readfirstlane(A.toff[y.s]);
    y.t1 = __builtin_amdgcn_readfirstlane(A.toff[y.s + 1]);
    y.nst = __builtin_amdgcn_readfirstlane(A.nstage[y.s]);
    y.ntot = uniform_d(A.n_species[y.c * A.S + y.s]);
    double* out = A.pops + y.c * A.N + y.base;
    if (!(y.ntot > 0.0)) {
      if (lane < y.Ns) out[lane] = 0.0;
      continue;
    }
    y.T = uniform_d(A.T_e[y.c]);
    y.ne = uniform_d(A.n_e[y.c]);
    y.kT = kBoltzmann * y.T;
    y.ikT = uniform_d(1.0 / y.kT);
    y.isqT = uniform_d(1.0 / sqrt(y.T));
    const double tfac = uniform_d(pow(y.T / 1e4, -0.8));
    for (int zz = 0; zz < 3; ++zz) {
      y.gion[zz] = uniform_d(A.gamma_ion[(y.c * A.S + y.s) * 3 + zz]);
      y.rec[zz] = uniform_d(y.ne * A.alpha0[y.s * 3 + zz] * tfac);
    }
    const bool live = lane < y.Ns;
    const int li = live ? y.base + lane : y.base;
    y.z = A.lv_ion[li];
    y.gnext = live ? A.lv_gnext[li] : -1;
    y.E = A.lv_E[li];
    y.g = A.lv_g[li];
    y.share = A.lv_share[li];
    y.rt = rt;

    double n = A.use_guess ? (live ? out[lane] : 0.0) : cold_start(y, live);
    if (A.use_guess && __ballot(live && !(n > 0.0 && n < INFINITY)) != 0ull)
      n = cold_start(y, live);  // unusable guess
    // From the guess (or the cold start) with the whole budget. With a warm
    // budget, a system still in its fixed-point phase or with a fixed-point
    // residual above 1e-6 after warm_budget iterations, or one whose line
    // search stalls, restarts once from the cold start with the iterations
    // left. One call site, so that the solver is compiled once.
    const bool checked = A.use_guess && A.warm_budget > 0 && A.warm_budget < A.max_iter;
    int its = -1, code = 0, spent = 0;
#pragma unroll 1
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (attempt == 1) {
        if (its >= 0 || !checked || spent >= A.max_iter) break;
        n = cold_start(y, live);
        code = 1;
      }
      int used = 0;
      its = solve_system<NT, NTB, MIX>(A, y, G, nb, hb, rowbuf, n, A.max_iter - spent,
                                  attempt == 0 && checked ? A.warm_budget : 0,
                                  attempt == 0 && A.use_guess, used);
      if (its >= 0) its += spent;
      spent += used;
    }
    if (live) out[lane] = n;
    if (lane == 0) {
      atomicMax(A.status + y.c, its < 0 ? 2 : code);
      if (A.iters) atomicMax(A.iters + y.c, its < 0 ? A.max_iter : its);
    }
  }
}

}  // namespace
}  // namespace extrass
