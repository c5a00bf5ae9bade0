/* Oracle copy of Philox4x64-10: counter-based generator of Salmon, Moraes,
 * Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).
 * Test infrastructure only (see oracle.h).
 *
 * One round maps the counter (x0,x1,x2,x3) with key (k0,k1) to
 *   (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0));
 * the key advances by the Weyl increments between rounds; ten rounds.
 */
#include "oracle.h"

static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mul128(PHILOX_M0, x0, &hi0, &lo0);
    mul128(PHILOX_M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}
