/*
 * Oracle (test infrastructure only): lozenge tilings of a general domain (the
 * domains of Section 1.1 on the triangular lattice of Section 1.2): a union of
 * unit triangles of the lattice Z^2 plus the diagonal (1,1), in the box of
 * w x h unit squares; heights H on its (w+1) x (h+1) vertices (index
 * Y*(w+1) + X); the sites are the vertices whose six triangles all belong to
 * the domain.  Same move, colouring and draws as the hexagon (lozenge.c): a
 * site is rotateable iff its forward neighbours (X+1,Y), (X,Y+1), (X+1,Y+1)
 * share a height f and its backward neighbours share f+1; up sets f+1;
 * colour (X + Y) mod 3; the draw of vertex (X, Y) is the site uniform of
 * (r, k) = (Y, X / 3).
 */
#include "oracle.h"

static int rotateable_r(int W, const int32_t *Hs, const uint8_t *site, int X, int Y, int32_t *f)
{
    int P = W + 1;
    if (!site[Y * P + X]) return 0;
    int32_t f1 = Hs[Y * P + X + 1], f2 = Hs[(Y + 1) * P + X], f3 = Hs[(Y + 1) * P + X + 1];
    int32_t b1 = Hs[Y * P + X - 1], b2 = Hs[(Y - 1) * P + X], b3 = Hs[(Y - 1) * P + X - 1];
    if (f1 != f2 || f1 != f3 || b1 != b2 || b1 != b3 || b1 != f1 + 1) return 0;
    *f = f1;
    return 1;
}

int or_lozr_flip(int W, int H, int32_t *Hs, const uint8_t *site, int X, int Y, int up)
{
    int32_t f;
    if (X < 1 || Y < 1 || X > W - 1 || Y > H - 1) return 0;
    if (!rotateable_r(W, Hs, site, X, Y, &f)) return 0;
    int32_t want = up ? f + 1 : f;
    if (Hs[Y * (W + 1) + X] == want) return 0;
    Hs[Y * (W + 1) + X] = want;
    return 1;
}

int or_lozr_sweeps(int W, int H, int32_t *Hs, const uint8_t *site, const uint32_t *thr, int metropolis,
                   uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours)
{
    int P = W + 1;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        uint32_t t = t0 + s;
        for (uint32_t i = 0; i < 3; ++i) {
            uint32_t step = 3u * t + i;
            int colour = random_colours ? (int)or_step_colour(seed, step, 3u) : (int)i;
            uint32_t tc = random_colours ? step : t;
            for (int Y = 1; Y < H; ++Y)
                for (int X = 1; X < W; ++X) {
                    if ((X + Y) % 3 != colour) continue;
                    int32_t f;
                    if (!rotateable_r(W, Hs, site, X, Y, &f)) continue;
                    int ctx = metropolis ? (Hs[Y * P + X] == f + 1) : 0;
                    uint32_t u = or_site_uniform(seed, (uint32_t)Y, (uint32_t)(X / 3), tc, (uint32_t)colour);
                    Hs[Y * P + X] = (u < thr[ctx]) ? f + 1 : f;
                }
        }
    }
    return 0;
}
