// Device-resident atom description shared by the NLTE, opacity and rate kernels.
#pragma once
#include <cstdint>
#include <vector>

#include "extrass.h"

namespace extrass {
constexpr int kMaxLevels = 64;  // one wavefront lane per level of a species
}

struct extrass_atom_ctx {
  int device = 0;
  int S = 0, N = 0, T = 0, maxNs = 0;
  int maxLine = -1;  // largest line index of a transition (trans_line)
  // stage blocks of the NLTE reduction (stage z's excited levels, its ground,
  // the next stage's ground): the largest block, and the most lanes a species'
  // blocks take side by side
  int maxBlock = 0, blockLanes = 0;
  // the NLTE matrix with rows packed to the levels each level couples to (its
  // stage, the next stage's ground, and for a ground the stage below): the
  // largest species' size in doubles
  int maxPacked = 0;
  std::vector<int> off;   // host copy of species_offset
  std::vector<int> toff;  // host: transitions of species s are [toff[s], toff[s+1])
  std::vector<double> lam_host;  // host copy of the transition wavelengths (caller's order)
  std::vector<int> lv_ion_host;   // host copy of each level's ion stage
  std::vector<double> lv_E_host;  // host copy of each level's energy above its stage's ground
  struct Dev {
    int32_t* off = nullptr;       // [S+1]
    int32_t* toff = nullptr;      // [S+1]
    int32_t* nstage = nullptr;    // [S]
    int32_t* lv_ion = nullptr;    // [N]
    int32_t* lv_gnext = nullptr;  // [N] local index of the next stage's ground, -1 if none
    double* lv_E = nullptr;       // [N]
    double* lv_g = nullptr;       // [N]
    double* lv_share = nullptr;   // [N] share of the recombination flux into the level
    // transitions grouped by species, for the NLTE assembly:
    // A lambda^3 / (8 pi), A, g_u/g_l, g_l/g_u, 8.629e-6 Upsilon / g_u, E_u - E_l
    double* t_pack = nullptr;     // [T*6]
    // local lower level, local upper level, caller's index (gamma_pe column), 0
    int32_t* t_idx = nullptr;     // [T*4]
    double* alpha0 = nullptr;     // [S*3]
    int32_t* o_lo = nullptr;      // [T] caller's order: global lower level
    int32_t* o_up = nullptr;
    int32_t* o_line = nullptr;
    double* o_A = nullptr;
    double* o_lam = nullptr;
    double* o_K = nullptr;         // [T] A lambda^3 / (8 pi) * g_u / g_l (Eq. A2 without n_l, t)
    double* o_r = nullptr;         // [T] g_l / g_u
  } d;
};
