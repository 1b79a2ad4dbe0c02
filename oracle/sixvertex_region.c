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
 * site code 2 marks a point on the free side of the domain (side 1 north,
 * 2 south, 3 east, 4 west).  It has no neighbour across that side; it flips
 * when its three other neighbours share a height m, with the context
 * (first diagonal at m+1) + 2 (second diagonal at m+1) of the free table, the
 * diagonals being the two points beside the two cells the flip changes:
 * north SW, SE; south NW, NE; east SW, NW; west SE, NE.  A domain with a free
 * south (west) side draws the uniform of point (I, J) as the point
 * (I + ox, J + oy) of the model's box, ox (oy) = 2, so that its free points
 * are inner points of that box; colours are unchanged (even offsets).
 */
#include "oracle.h"

static int flippable_r(int W, const int32_t *h, const uint8_t *site, int side, int I, int J, int32_t *m,
                       unsigned *mask)
{
    int P = W + 1;
    if (!site[J * P + I]) return 0;
    if (site[J * P + I] == 2) {   /* a free point: three neighbours, two diagonal points */
        int32_t a, b, c;
        const int32_t *d0, *d1;
        switch (side) {
        case 1:   /* north: W, E, S; diagonals SW, SE */
            a = h[J * P + I - 1]; b = h[J * P + I + 1]; c = h[(J - 1) * P + I];
            d0 = &h[(J - 1) * P + I - 1]; d1 = &h[(J - 1) * P + I + 1];
            break;
        case 2:   /* south: W, E, N; diagonals NW, NE */
            a = h[J * P + I - 1]; b = h[J * P + I + 1]; c = h[(J + 1) * P + I];
            d0 = &h[(J + 1) * P + I - 1]; d1 = &h[(J + 1) * P + I + 1];
            break;
        case 3:   /* east: W, N, S; diagonals SW, NW */
            a = h[J * P + I - 1]; b = h[(J + 1) * P + I]; c = h[(J - 1) * P + I];
            d0 = &h[(J - 1) * P + I - 1]; d1 = &h[(J + 1) * P + I - 1];
            break;
        case 4:   /* west: E, N, S; diagonals SE, NE */
            a = h[J * P + I + 1]; b = h[(J + 1) * P + I]; c = h[(J - 1) * P + I];
            d0 = &h[(J - 1) * P + I + 1]; d1 = &h[(J + 1) * P + I + 1];
            break;
        default:
            return 0;
        }
        if (a != b || a != c) return 0;
        *m = a;
        *mask = (*d0 == a + 1 ? 1u : 0u) | (*d1 == a + 1 ? 2u : 0u);
        return 1;
    }
    int32_t e = h[J * P + I + 1], w = h[J * P + I - 1], s = h[(J - 1) * P + I];
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

int or_sixvr_flip(int W, int H, int32_t *h, const uint8_t *site, int side, int I, int J, int up)
{
    int32_t m;
    unsigned mask;
    if (I < 0 || J < 0 || I > W || J > H) return 0;
    if (!flippable_r(W, h, site, side, I, J, &m, &mask)) return 0;
    int32_t want = up ? m + 1 : m - 1;
    if (h[J * (W + 1) + I] == want) return 0;
    h[J * (W + 1) + I] = want;
    return 1;
}

int or_sixvr_sweeps(int W, int H, int32_t *h, const uint8_t *site, const uint32_t *thr, const uint32_t *thr_free,
                    int metropolis, uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, int side,
                    int ox, int oy)
{
    int P = W + 1;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        uint32_t t = t0 + s;
        for (uint32_t i = 0; i < 4; ++i) {
            uint32_t step = 4u * t + i;
            int colour = random_colours ? (int)or_step_colour(seed, step, 4u) : (int)i;
            uint32_t tc = random_colours ? step : t;
            for (int J = 0; J <= H; ++J)
                for (int I = 0; I <= W; ++I) {
                    if ((I & 1) + 2 * (J & 1) != colour) continue;
                    int32_t m;
                    unsigned mask;
                    if (!flippable_r(W, h, site, side, I, J, &m, &mask)) continue;
                    unsigned ctx = metropolis ? 2u * mask + (h[J * P + I] == m + 1) : mask;
                    const uint32_t *T = site[J * P + I] == 2 ? thr_free : thr;
                    uint32_t u = or_site_uniform(seed, (uint32_t)(J + oy), (uint32_t)((I + ox) >> 1), tc,
                                                 (uint32_t)colour);
                    h[J * P + I] = (u < T[ctx]) ? m + 1 : m - 1;
                }
        }
    }
    return 0;
}
