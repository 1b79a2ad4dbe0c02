/*
 * Oracle (test infrastructure only): Philox4x32-10 and the per-site uniform.
 *
 * Philox4x32 follows Salmon, Moraes, Dror and Shaw, "Parallel Random Numbers:
 * As Easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 multiplications
 * with the published multipliers, the key bumped by the published Weyl
 * constants between rounds.  The paper itself draws with TinyMT (Section 2.2.1);
 * a counter-based generator replaces it so that every draw is a pure function of
 * (seed, sweep, colour, site), see the conventions in the design notes.
 */
#include "oracle.h"

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The uniform u of the site with class coordinates (r, k) in colour step
 * (sweep t, colour c).  Bit (31-j) of u, i.e. plane j counted from the most
 * significant bit, is bit (k & 31) of output word (k >> 5) & 3 of Philox with
 * counter (k >> 7, r, t, 4j + c).  All 32 planes are generated: the oracle does
 * not shortcut the comparison u < T. */
uint32_t or_site_uniform(uint64_t seed, uint32_t r, uint32_t k, uint32_t t, uint32_t c)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t u = 0;
    for (uint32_t j = 0; j < 32; ++j) {
        uint32_t ctr[4] = {k >> 7, r, t, (j << 2) | c};
        uint32_t out[4];
        or_philox4x32_10(ctr, key, out);
        uint32_t bit = (out[(k >> 5) & 3u] >> (k & 31u)) & 1u;
        u |= bit << (31u - j);
    }
    return u;
}

/* Iteration order switch used by the order-independence tests. */
/* Colour of colour step `step` under the random colour order: the paper's
 * RandomWalk picks the colour of every step at random; here it is
 * floor(K u / 2^32) with u word 0 of Philox(key = seed, ctr = (step, 0, 0, 2^31)),
 * a counter no site draw uses (their last word is below 128). */
uint32_t or_step_colour(uint64_t seed, uint32_t step, uint32_t K)
{
    const uint32_t ctr[4] = {step, 0u, 0u, 0x80000000u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return (uint32_t)(((uint64_t)out[0] * K) >> 32);
}

int or_reverse_order = 0;
void or_set_reverse_order(int reverse) { or_reverse_order = reverse ? 1 : 0; }
