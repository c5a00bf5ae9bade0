/* Oracle: photoionising levels and their cross sections (Sec. 2.3.1; Eq. A5).
 * Test infrastructure only (see oracle.h). FP64.
 *
 * The paper photoionises from neutral and singly ionised stages only (no
 * ionisation from the doubly ionised stage upwards), from a per-ion number of
 * the lowest levels, with the hydrogenic cross section of Eq. A5 for excited
 * states (Verner fits for ground states and TOPBASE data for a few levels are
 * not available here, so every level takes the hydrogenic form):
 *   sigma(lambda) = 7.9e-18 cm^2 (lambda / lambda_i)^3 (1 - E_i / E_ion)^-1/2 / (z + 1)^2
 * for lambda <= lambda_i = h c / (E_ion - E_i), zero redward of the threshold.
 * E_i is the level's energy above its stage's ground, E_ion the stage's
 * ionisation energy, z the stage's charge.
 */
#include <math.h>

#include "oracle.h"

#define HC_ERG_CM (6.62607015e-27 * 2.99792458e10)
#define SIGMA_KRAMERS 7.9e-18 /* cm^2, Eq. A5 */

int32_t oracle_pi_levels(const or_atom* a, const double* ion_energy, int32_t max_per_stage,
                         int32_t* level, double* lambda_thr, double* sigma0) {
  int32_t m = 0;
  for (int32_t s = 0; s < a->n_species; ++s) {
    const int32_t b = a->species_offset[s], e = a->species_offset[s + 1];
    int32_t top = 0;
    for (int32_t i = b; i < e; ++i)
      if (a->level_ion[i] > top) top = a->level_ion[i];
    for (int32_t z = 0; z < 2 && z < top; ++z) {
      const double E_ion = ion_energy[s * 3 + z];
      int32_t taken = 0;
      for (int32_t i = b; i < e && taken < max_per_stage; ++i) {
        if (a->level_ion[i] != z) continue;
        const double chi = E_ion - a->level_energy[i];
        if (!(chi > 0.0)) continue; /* not bound below the stage's threshold */
        ++taken;
        if (level) level[m] = i;
        if (lambda_thr) lambda_thr[m] = HC_ERG_CM / chi;
        if (sigma0) sigma0[m] = SIGMA_KRAMERS / sqrt(chi / E_ion) / ((z + 1.0) * (z + 1.0));
        ++m;
      }
    }
  }
  return m;
}
