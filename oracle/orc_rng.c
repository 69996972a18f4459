/*
 * AIRPF CPU oracle -- Philox4x32-10 and the draw layout.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
 *   (c0,c1,c2,c3) <- (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
 * with M0 = 0xD2511F53, M1 = 0xCD9E8D57, the key bumped by the Weyl constants
 * (0x9E3779B9, 0xBB67AE85) between rounds.
 *
 * Draw layout (the random numbers the filter consumes; Algorithm 1 leaves
 * their source open):
 *   key     = (seed mod 2^32, seed >> 32)
 *   counter = (c0, c1 = island k, c2 = step n, c3 = tag << 24 | sub)
 *   NORMAL : c0 = e >> 2 for normal e = j*dx + d of (step n, island k);
 *            words (w0,w1) -> normals 4g, 4g+1; (w2,w3) -> 4g+2, 4g+3.
 *            Step 0 draws initialise, step n >= 1 draws mutate into step n.
 *   SYS    : c0 = 0: the systematic offset of island k at step n.
 *   MULT   : c0 = j: the j-th multinomial draw of island k at step n.
 *   ISL    : c0 = s: the pair-selection uniform of island k, stage s, step n.
 *   BIN    : c0 = j: word 0 drives particle j of the binary model.
 *   BCP    : c0 = 2j + b (b = 0, 1): the eight words of particle j of the
 *            Beta change-point model.
 *   BIN    : c0 = j: the binary toy model's per-particle word.
 *   sub    : 0, 1, ... extra blocks for rejection retries.
 */
#include <stdint.h>
#include "orc.h"

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
              uint32_t tag, uint32_t sub, uint32_t w[4]) {
  const uint32_t ctr[4] = {c0, c1, c2, (tag << 24) | (sub & 0xffffffu)};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox(ctr, key, w);
}

/* uniform on [0,1) with 53 random bits: x = hi*2^32 + lo, u = (x >> 11) 2^-53 */
double orc_u53(uint32_t hi, uint32_t lo) {
  const uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
  return (double)(x >> 11) * 0x1p-53;
}

/* Uniform integer on [0, Q), Q >= 1, by Lemire's multiply-and-reject method
 * ("Fast random integer generation in an interval", ACM TOMACS 2019):
 * candidate x (64 bits); p = x*Q (128 bits); accept unless
 * (p mod 2^64) < (2^64 mod Q); result p >> 64.  Candidates are taken in the
 * order (w0,w1), (w2,w3) of sub-block 0, then sub-block 1, ...  After 64
 * sub-blocks (probability below 2^-1600 for Q < 2^52) the last candidate is
 * returned as is. */
uint64_t orc_bounded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                     uint32_t tag, uint64_t Q) {
  const uint64_t thresh = (0 - Q) % Q;                 /* 2^64 mod Q         */
  uint64_t result = 0;
  for (uint32_t sub = 0; sub < 64; ++sub) {
    uint32_t w[4];
    orc_draw(seed, c0, c1, c2, tag, sub, w);
    for (int h = 0; h < 2; ++h) {
      const uint64_t x = ((uint64_t)w[2 * h] << 32) | (uint64_t)w[2 * h + 1];
      const unsigned __int128 p = (unsigned __int128)x * (unsigned __int128)Q;
      result = (uint64_t)(p >> 64);
      if ((uint64_t)p >= thresh) return result;
    }
  }
  return result;
}

/* normals e = 0 .. count-1 of (step n, island k) */
void orc_island_normals(uint64_t seed, int64_t n, int32_t k, int64_t count,
                        double* z) {
  for (int64_t g = 0; 4 * g < count; ++g) {
    uint32_t w[4];
    orc_draw(seed, (uint32_t)g, (uint32_t)k, (uint32_t)n, TAG_NORMAL, 0, w);
    double t[4];
    orc_boxmuller(w[0], w[1], &t[0], &t[1]);
    orc_boxmuller(w[2], w[3], &t[2], &t[3]);
    for (int r = 0; r < 4 && 4 * g + r < count; ++r) z[4 * g + r] = t[r];
  }
}

/* the same normals in binary32 arithmetic (orc_boxmullerf), stored widened */
void orc_island_normalsf(uint64_t seed, int64_t n, int32_t k, int64_t count,
                         double* z) {
  for (int64_t g = 0; 4 * g < count; ++g) {
    uint32_t w[4];
    orc_draw(seed, (uint32_t)g, (uint32_t)k, (uint32_t)n, TAG_NORMAL, 0, w);
    float t[4];
    orc_boxmullerf(w[0], w[1], &t[0], &t[1]);
    orc_boxmullerf(w[2], w[3], &t[2], &t[3]);
    for (int r = 0; r < 4 && 4 * g + r < count; ++r) z[4 * g + r] = (double)t[r];
  }
}
