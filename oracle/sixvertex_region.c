/*
 * Oracle (test infrastructure only): the six-vertex model on a general domain
 * (Section 1.2, with the domains of Section 1.1): the vertices of the model are
 * the cells of a mask, the heights live on the (W+1) x (H+1) corner points of
 * the W x H cell box (point (I, J) at index J*(W+1) + I), and the sites are the
 * points whose four cells all belong to the domain.  Heights on the other
 * points of the domain are fixed by its boundary.
 *
 * Same move, colouring, contexts and draws as the domain-wall square
 * (sixvertex.c): a site is flippable iff its four edge-neighbours share a
 * height m; up sets m+1, down m-1; colour (I mod 2) + 2 (J mod 2); the draw of
 * point (I, J) is the site uniform of (r, k) = (J, I >> 1).
 *
 * Free boundary (the variation of c-flips for boundary faces of Section 1.2):
 * site code 2 marks a point on a free north edge of the domain.  It has no
 * north neighbour; it flips when its west, east and south neighbours share a
 * height m, with the context (SW at m+1) + 2 (SE at m+1) of the free table.
 */
#include "oracle.h"

static int flippable_r(int W, const int32_t *h, const uint8_t *site, int I, int J, int32_t *m, unsigned *mask)
{
    int P = W + 1;
    if (!site[J * P + I]) return 0;
    int32_t e = h[J * P + I + 1], w = h[J * P + I - 1], s = h[(J - 1) * P + I];
    if (site[J * P + I] == 2) {   /* free north edge: three neighbours, two diagonal faces */
        if (e != w || e != s) return 0;
        *m = e;
        *mask = (h[(J - 1) * P + I - 1] == e + 1 ? 1u : 0u) | (h[(J - 1) * P + I + 1] == e + 1 ? 2u : 0u);
        return 1;
    }
    int32_t nn = h[(J + 1) * P + I];
    if (e != w || e != nn || e != s) return 0;
    *m = e;
    unsigned k = 0;
    if (h[(J + 1) * P + I + 1] == e + 1) k |= 1u;
    if (h[(J + 1) * P + I - 1] == e + 1) k |= 2u;
    if (h[(J - 1) * P + I - 1] == e + 1) k |= 4u;
    if (h[(J - 1) * P + I + 1] == e + 1) k |= 8u;
    *mask = k;
    return 1;
}

int or_sixvr_flip(int W, int H, int32_t *h, const uint8_t *site, int I, int J, int up)
{
    int32_t m;
    unsigned mask;
    if (I < 1 || J < 1 || I > W - 1 || J > H) return 0;
    if (!flippable_r(W, h, site, I, J, &m, &mask)) return 0;
    int32_t want = up ? m + 1 : m - 1;
    if (h[J * (W + 1) + I] == want) return 0;
    h[J * (W + 1) + I] = want;
    return 1;
}

int or_sixvr_sweeps(int W, int H, int32_t *h, const uint8_t *site, const uint32_t *thr, const uint32_t *thr_free,
                    int metropolis, uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours)
{
    int P = W + 1;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        uint32_t t = t0 + s;
        for (uint32_t i = 0; i < 4; ++i) {
            uint32_t step = 4u * t + i;
            int colour = random_colours ? (int)or_step_colour(seed, step, 4u) : (int)i;
            uint32_t tc = random_colours ? step : t;
            for (int J = 1; J <= H; ++J)
                for (int I = 1; I < W; ++I) {
                    if ((I & 1) + 2 * (J & 1) != colour) continue;
                    int32_t m;
                    unsigned mask;
                    if (!flippable_r(W, h, site, I, J, &m, &mask)) continue;
                    unsigned ctx = metropolis ? 2u * mask + (h[J * P + I] == m + 1) : mask;
                    const uint32_t *T = site[J * P + I] == 2 ? thr_free : thr;
                    uint32_t u = or_site_uniform(seed, (uint32_t)J, (uint32_t)(I >> 1), tc, (uint32_t)colour);
                    h[J * P + I] = (u < T[ctx]) ? m + 1 : m - 1;
                }
        }
    }
    return 0;
}
