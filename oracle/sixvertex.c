/*
 * Oracle (test infrastructure only): six-vertex model on the N x N grid with
 * domain-wall boundary conditions.
 *
 * Section 1.2 (The six-vertex model): configurations are in bijection with
 * height functions on faces (Figure "sixvertexh": crossing an occupied vertical
 * edge in +x adds 1, an empty one subtracts 1; likewise for horizontal edges in
 * +y).  The set of configurations with fixed boundary is connected by c-flips at
 * faces; cluster moves colour faces by the parities of both coordinates.  A
 * configuration has the weight prod_v w(v), with a, b, c the weights of the
 * a-, b-, c-type vertices of Figure "sixvertex"(A).
 *
 * Readings (listed in the design notes): faces (I, J), 0 <= I, J <= N, the
 * outer ring fixed by the domain-wall boundary h(I,0) = I, h(0,J) = J,
 * h(I,N) = N-I, h(N,J) = N-J (all legs on the south and west sides occupied).
 * An interior face is flippable iff its four edge-neighbours share a height m;
 * it then takes m+1 (up) or m-1.  The vertex at a corner of the face is of type
 * c iff both diagonal pairs of its four faces are equal; otherwise it is of type
 * a when the face and its diagonal are the south-west/north-east pair of that
 * vertex (corners NE and SW of the face) and of type b otherwise (NW and SE).
 * Colour = (I mod 2) + 2 (J mod 2).
 */
#include <stdlib.h>
#include "oracle.h"

static int iabs(int v) { return v < 0 ? -v : v; }

void or_sixv_min(int N, int32_t *h)
{
    for (int J = 0; J <= N; ++J)
        for (int I = 0; I <= N; ++I) h[J * (N + 1) + I] = iabs(I - J);
}

void or_sixv_max(int N, int32_t *h)
{
    for (int J = 0; J <= N; ++J)
        for (int I = 0; I <= N; ++I) h[J * (N + 1) + I] = N - iabs(I + J - N);
}

/* If face (I, J) is flippable, return 1 with the neighbour height m and the
 * mask of diagonal faces at height m+1 (NE=1, NW=2, SW=4, SE=8). */
static int flippable(int N, const int32_t *h, int I, int J, int32_t *m, unsigned *mask)
{
    int P = N + 1;
    if (I < 1 || J < 1 || I > N - 1 || J > N - 1) return 0;
    int32_t e = h[J * P + I + 1], w = h[J * P + I - 1], nn = h[(J + 1) * P + I], s = h[(J - 1) * P + I];
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

int or_sixv_flip(int N, int32_t *h, int I, int J, int up)
{
    int32_t m;
    unsigned mask;
    if (!flippable(N, h, I, J, &m, &mask)) return 0;
    int32_t want = up ? m + 1 : m - 1;
    if (h[J * (N + 1) + I] == want) return 0;
    h[J * (N + 1) + I] = want;
    return 1;
}

int64_t or_sixv_observe(int N, const int32_t *h, uint32_t bin, uint64_t *bin_sum)
{
    int P = N + 1;
    int bx = (N + (int)bin - 1) / (int)bin;
    int64_t count = 0;
    for (int j = 1; j <= N; ++j)
        for (int i = 1; i <= N; ++i) {
            int isc = h[(j - 1) * P + i - 1] == h[j * P + i] && h[(j - 1) * P + i] == h[j * P + i - 1];
            if (!isc) continue;
            ++count;
            if (bin_sum) bin_sum[((j - 1) / (int)bin) * bx + (i - 1) / (int)bin] += 1;
        }
    return count;
}

int or_sixv_sweeps(int N, int32_t *h, const uint32_t *thr, int metropolis,
                   uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, or_obs *obs)
{
    int P = N + 1;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        uint32_t t = t0 + s;
        for (uint32_t i = 0; i < 4; ++i) {
            /* the colour of the step and the sweep counter of its draws */
            uint32_t step = 4u * t + i;
            int colour = random_colours ? (int)or_step_colour(seed, step, 4u) : (int)i;
            uint32_t tc = random_colours ? step : t;
            for (int Ji = 1; Ji < N; ++Ji)
                for (int Ii = 1; Ii < N; ++Ii) {
                    int J = or_reverse_order ? N - Ji : Ji;
                    int I = or_reverse_order ? N - Ii : Ii;
                    if ((I & 1) + 2 * (J & 1) != colour) continue;
                    int32_t m;
                    unsigned mask;
                    if (!flippable(N, h, I, J, &m, &mask)) continue;
                    unsigned ctx = metropolis ? 2u * mask + (h[J * P + I] == m + 1) : mask;
                    uint32_t u = or_site_uniform(seed, (uint32_t)J, (uint32_t)(I >> 1), tc,
                                                 (uint32_t)colour);
                    h[J * P + I] = (u < thr[ctx]) ? m + 1 : m - 1;
                }
        }
        if (obs && obs->obs_every && (t + 1) % obs->obs_every == 0) {
            int64_t v = or_sixv_observe(N, h, obs->bin, obs->bin_sum);
            if (obs->scalar_sum) *obs->scalar_sum += v;
            if (obs->samples) *obs->samples += 1;
        }
    }
    return 0;
}
