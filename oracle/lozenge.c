/*
 * Oracle (test infrastructure only): lozenge tilings of the a x b x c hexagon.
 *
 * Section 1.2 (Lozenge tilings): lozenge tilings are dimers on the hexagonal
 * lattice; their height function lives on the vertices of the triangular
 * lattice; elementary rotations act at triangular vertices; clusters come from a
 * 3-colouring of the triangular lattice.  Volume weights (Section 1.1.1) give a
 * tiling the weight q^volume.
 *
 * Readings (listed in the design notes): the triangular lattice is Z^2 with the
 * extra diagonal (1,1); the height H is the number of unit cubes of the boxed
 * plane partition on the lattice line through the vertex, so along each of the
 * directions (1,0), (0,1), (1,1) H changes by 0 or -1.  The hexagon is the set
 * -c <= x <= a, -c <= y <= b, -b <= x - y <= a; H_min = max(0, -x, -y) is the
 * empty box, H_max = min(c, a-x, b-y) the full one.  A vertex is rotateable iff
 * its three forward neighbours share a height f and its three backward
 * neighbours share f+1; the up-rotation (adding a cube) sets H = f+1.
 * Colour = (X + Y) mod 3 in shifted coordinates X = x + c, Y = y + c.
 */
#include <limits.h>
#include <stdlib.h>
#include "oracle.h"

int or_lozenge_box(int a, int b, int c, int *W, int *H)
{
    *W = a + c + 1;
    *H = b + c + 1;
    return (*W) * (*H);
}

static int in_hex(int a, int b, int c, int X, int Y)
{
    int x = X - c, y = Y - c;
    return x >= -c && x <= a && y >= -c && y <= b && x - y >= -b && x - y <= a;
}

static int interior(int a, int b, int c, int X, int Y)
{
    int x = X - c, y = Y - c;
    return x > -c && x < a && y > -c && y < b && x - y > -b && x - y < a;
}

static int imax3(int p, int q, int r) { int m = p > q ? p : q; return m > r ? m : r; }
static int imin3(int p, int q, int r) { int m = p < q ? p : q; return m < r ? m : r; }

static int hmin(int c, int X, int Y) { return imax3(0, -(X - c), -(Y - c)); }

void or_lozenge_min(int a, int b, int c, int32_t *Hs)
{
    int W = a + c + 1, Hh = b + c + 1;
    for (int Y = 0; Y < Hh; ++Y)
        for (int X = 0; X < W; ++X)
            Hs[Y * W + X] = in_hex(a, b, c, X, Y) ? hmin(c, X, Y) : INT32_MIN;
}

void or_lozenge_max(int a, int b, int c, int32_t *Hs)
{
    int W = a + c + 1, Hh = b + c + 1;
    for (int Y = 0; Y < Hh; ++Y)
        for (int X = 0; X < W; ++X) {
            int x = X - c, y = Y - c;
            Hs[Y * W + X] = in_hex(a, b, c, X, Y) ? imin3(c, a - x, b - y) : INT32_MIN;
        }
}

/* If the site is rotateable, return 1 and the forward height f. */
static int hexagon_at(int a, int b, int c, const int32_t *Hs, int X, int Y, int32_t *f)
{
    int W = a + c + 1;
    if (!interior(a, b, c, X, Y)) return 0;
    int32_t f1 = Hs[Y * W + X + 1], f2 = Hs[(Y + 1) * W + X], f3 = Hs[(Y + 1) * W + X + 1];
    int32_t b1 = Hs[Y * W + X - 1], b2 = Hs[(Y - 1) * W + X], b3 = Hs[(Y - 1) * W + X - 1];
    if (f1 != f2 || f1 != f3 || b1 != b2 || b1 != b3 || b1 != f1 + 1) return 0;
    *f = f1;
    return 1;
}

int or_lozenge_flip(int a, int b, int c, int32_t *Hs, int X, int Y, int up)
{
    int W = a + c + 1;
    int32_t f;
    if (!hexagon_at(a, b, c, Hs, X, Y, &f)) return 0;
    int32_t want = up ? f + 1 : f;
    if (Hs[Y * W + X] == want) return 0;
    Hs[Y * W + X] = want;
    return 1;
}

int64_t or_lozenge_observe(int a, int b, int c, const int32_t *Hs, uint32_t bin, uint64_t *bin_sum)
{
    int W = a + c + 1, Hh = b + c + 1;
    int bx = (W + (int)bin - 1) / (int)bin;
    int64_t vol = 0;
    for (int Y = 0; Y < Hh; ++Y)
        for (int X = 0; X < W; ++X) {
            if (!in_hex(a, b, c, X, Y)) continue;
            int64_t q = (int64_t)Hs[Y * W + X] - hmin(c, X, Y);
            vol += q;
            if (bin_sum) bin_sum[(Y / (int)bin) * bx + X / (int)bin] += (uint64_t)q;
        }
    return vol;
}

int or_lozenge_sweeps(int a, int b, int c, int32_t *Hs, const uint32_t *thr, int metropolis,
                      uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, or_obs *obs)
{
    int W = a + c + 1, Hh = b + c + 1;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        uint32_t t = t0 + s;
        for (uint32_t i = 0; i < 3; ++i) {
            /* the colour of the step and the sweep counter of its draws */
            uint32_t step = 3u * t + i;
            int colour = random_colours ? (int)or_step_colour(seed, step, 3u) : (int)i;
            uint32_t tc = random_colours ? step : t;
            for (int Yi = 0; Yi < Hh; ++Yi)
                for (int Xi = 0; Xi < W; ++Xi) {
                    int Y = or_reverse_order ? Hh - 1 - Yi : Yi;
                    int X = or_reverse_order ? W - 1 - Xi : Xi;
                    if ((X + Y) % 3 != colour) continue;
                    int32_t f;
                    if (!hexagon_at(a, b, c, Hs, X, Y, &f)) continue;
                    int ctx = metropolis ? (Hs[Y * W + X] == f + 1) : 0;
                    uint32_t u = or_site_uniform(seed, (uint32_t)Y, (uint32_t)(X / 3), tc,
                                                 (uint32_t)colour);
                    Hs[Y * W + X] = (u < thr[ctx]) ? f + 1 : f;
                }
        }
        if (obs && obs->obs_every && (t + 1) % obs->obs_every == 0) {
            int64_t v = or_lozenge_observe(a, b, c, Hs, obs->bin, obs->bin_sum);
            if (obs->scalar_sum) *obs->scalar_sum += v;
            if (obs->samples) *obs->samples += 1;
        }
    }
    return 0;
}
