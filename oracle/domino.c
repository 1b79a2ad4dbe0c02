/*
 * Oracle (test infrastructure only): domino tilings of the Aztec diamond.
 *
 * Follows Section 2.2 of the paper step by step:
 *   - every vertex v carries the tilestate s_v = e0 + 2 e1 + 4 e2 + 8 e3 over its
 *     edges North, South, East, West (e_i = 1 when a domino crosses the edge);
 *     v is rotateable iff s_v is 3 (two horizontal dominoes) or 12 (two vertical);
 *   - the N x N array T is split into the black array T_b, T_b[i,j] <-> vertex
 *     (i, 2j + i mod 2), and the white array T_w, T_w[i,j] <-> (i, 2j + 1 - i mod 2),
 *     both zero padded;
 *   - a colour step runs Rotate on one array (each rotateable vertex becomes 12
 *     or 3 according to its draw; an up-rotation turns the horizontal pair into
 *     the vertical pair, Section 1.1.2) and then Update on the other array with
 *     the bitwise formula of Section 2.2 (UpdateWhite is the same formula with
 *     the roles of the arrays exchanged).
 *
 * Readings taken where the paper is silent or ambiguous (listed in the design
 * notes): the paper's matrix rows run north to south and its columns run west
 * to east-mirrored, i.e. its "East" bit 4 refers to the neighbour at column-1;
 * here the box vertex (X, Y), X eastward and Y northward, sits at row 2n+1-Y
 * and column 2n+1-X, so bit 4 is the geometric east edge.  Colours are visited
 * in the fixed order black (x+y even) then white in every sweep, instead of the
 * paper's coin flip per step.  The heat-bath rule (Section 1.1.1 weights):
 * a rotateable vertex becomes vertical iff u < thr[ctx].
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define S_N 1u
#define S_S 2u
#define S_E 4u
#define S_W 8u

static int dim(int n) { return 2 * n + 4; }          /* N: even, padded */
int or_domino_array_len(int n) { return dim(n) * (dim(n) / 2); }

static uint8_t get(const uint8_t *T, int n, int i, int j)
{
    int N = dim(n);
    if (i < 0 || i >= N || j < 0 || j >= N / 2) return 0;
    return T[i * (N / 2) + j];
}

/* UpdateBlack of Section 2.2: recompute T_b from T_w. */
static void update_black(int n, uint8_t *Tb, const uint8_t *Tw)
{
    int N = dim(n), M = N / 2;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < M; ++j) {
            int p = i & 1;
            unsigned s = (get(Tw, n, i - 1, j) & 2u) / 2u + 2u * (get(Tw, n, i + 1, j) & 1u) +
                         (get(Tw, n, i, j + p - 1) & 8u) / 2u + 2u * (get(Tw, n, i, j + p) & 4u);
            Tb[i * M + j] = (uint8_t)s;
        }
}

/* UpdateWhite: the same formula for T_w[i,j] <-> (i, 2j + 1 - i mod 2). */
static void update_white(int n, uint8_t *Tw, const uint8_t *Tb)
{
    int N = dim(n), M = N / 2;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < M; ++j) {
            int p = i & 1;
            unsigned s = (get(Tb, n, i - 1, j) & 2u) / 2u + 2u * (get(Tb, n, i + 1, j) & 1u) +
                         (get(Tb, n, i, j - p) & 8u) / 2u + 2u * (get(Tb, n, i, j + 1 - p) & 4u);
            Tw[i * M + j] = (uint8_t)s;
        }
}

/* Location of box vertex (X, Y), X, Y in [0, 2n], in the split arrays. */
static uint8_t *vertex_slot(int n, uint8_t *Tb, uint8_t *Tw, int X, int Y)
{
    int M = dim(n) / 2;
    int i = 2 * n + 1 - Y, col = 2 * n + 1 - X;
    if ((X + Y) % 2 == 0) return &Tb[i * M + (col - (i & 1)) / 2];
    return &Tw[i * M + (col - 1 + (i & 1)) / 2];
}

static uint8_t vertex_state(int n, const uint8_t *Tb, const uint8_t *Tw, int X, int Y)
{
    if (X < 0 || Y < 0 || X > 2 * n || Y > 2 * n) return 0;
    return *vertex_slot(n, (uint8_t *)Tb, (uint8_t *)Tw, X, Y);
}

int or_domino_vertex_state(int n, const uint8_t *Tb, const uint8_t *Tw, int X, int Y)
{
    return vertex_state(n, Tb, Tw, X, Y);
}

static int face_in(int n, int X, int Y)
{
    if (X < 0 || Y < 0 || X >= 2 * n || Y >= 2 * n) return 0;
    return abs(2 * X - 2 * n + 1) + abs(2 * Y - 2 * n + 1) <= 2 * n;
}

int or_domino_from_faces(int n, const uint8_t *faces, uint8_t *Tb, uint8_t *Tw, int allow_uncovered)
{
    int W = 2 * n;
    memset(Tb, 0, (size_t)or_domino_array_len(n));
    memset(Tw, 0, (size_t)or_domino_array_len(n));
    for (int Y = 0; Y < W; ++Y)
        for (int X = 0; X < W; ++X) {
            uint8_t d = faces[Y * W + X];
            if (!face_in(n, X, Y)) {
                if (d != 0xFF) return -1;
                continue;
            }
            /* a region inside the diamond: faces outside it stay uncovered */
            if (allow_uncovered && d == 0xFF) continue;
            int PX = X + (d == 2) - (d == 3), PY = Y + (d == 0) - (d == 1);
            if (d > 3 || !face_in(n, PX, PY)) return -1;
            uint8_t back = faces[PY * W + PX];
            if (back != (uint8_t)(d ^ 1u)) return -1;   /* N<->S, E<->W */
            if (d == 2) {            /* crossed edge (X+1,Y)-(X+1,Y+1) */
                *vertex_slot(n, Tb, Tw, X + 1, Y) |= S_N;
                *vertex_slot(n, Tb, Tw, X + 1, Y + 1) |= S_S;
            } else if (d == 0) {     /* crossed edge (X,Y+1)-(X+1,Y+1) */
                *vertex_slot(n, Tb, Tw, X, Y + 1) |= S_E;
                *vertex_slot(n, Tb, Tw, X + 1, Y + 1) |= S_W;
            }
        }
    return 0;
}

void or_domino_to_faces(int n, const uint8_t *Tb, const uint8_t *Tw, uint8_t *faces)
{
    int W = 2 * n;
    for (int Y = 0; Y < W; ++Y)
        for (int X = 0; X < W; ++X) {
            uint8_t d = 0xFF;
            if (face_in(n, X, Y)) {
                if (vertex_state(n, Tb, Tw, X, Y + 1) & S_E) d = 0;        /* top edge */
                else if (vertex_state(n, Tb, Tw, X, Y) & S_E) d = 1;       /* bottom edge */
                else if (vertex_state(n, Tb, Tw, X + 1, Y) & S_N) d = 2;   /* right edge */
                else if (vertex_state(n, Tb, Tw, X, Y) & S_N) d = 3;       /* left edge */
            }
            faces[Y * W + X] = d;
        }
}

/* All-horizontal brick tiling: every face row of the diamond (an even number of
 * faces) is covered by horizontal dominoes starting at its west end. */
void or_domino_brick(int n, uint8_t *Tb, uint8_t *Tw)
{
    int W = 2 * n;
    uint8_t *faces = (uint8_t *)malloc((size_t)W * W);
    for (int Y = 0; Y < W; ++Y) {
        int start = -1;
        for (int X = 0; X < W; ++X) {
            if (!face_in(n, X, Y)) { faces[Y * W + X] = 0xFF; continue; }
            if (start < 0) start = X;
            faces[Y * W + X] = ((X - start) % 2 == 0) ? 2 : 3;
        }
    }
    or_domino_from_faces(n, faces, Tb, Tw, 0);
    free(faces);
}

int or_domino_flip(int n, uint8_t *Tb, uint8_t *Tw, int X, int Y, int up)
{
    if (X < 0 || Y < 0 || X > 2 * n || Y > 2 * n) return 0;
    uint8_t *s = vertex_slot(n, Tb, Tw, X, Y);
    if (*s != 3 && *s != 12) return 0;
    uint8_t want = up ? 12 : 3;
    if (*s == want) return 0;
    *s = want;
    if ((X + Y) % 2 == 0) update_white(n, Tw, Tb);
    else update_black(n, Tb, Tw);
    return 1;
}

static int mod2(int v) { return ((v % 2) + 2) % 2; }
static int floordiv2(int v) { return (v >= 0) ? v / 2 : -((-v + 1) / 2); }

/* Rotate of Section 2.2 on the array of colour c. */
static void rotate(int n, uint8_t *T, int colour, const uint32_t *thr, int metropolis,
                   uint64_t seed, uint32_t t)
{
    int N = dim(n), M = N / 2;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < M; ++j) {
            uint8_t s = T[i * M + j];
            if (s != 3 && s != 12) continue;
            int col = colour == 0 ? 2 * j + (i & 1) : 2 * j + 1 - (i & 1);
            int X = 2 * n + 1 - col, Y = 2 * n + 1 - i;
            int x = X - n, y = Y - n;
            uint32_t r = (uint32_t)floordiv2(x + y + n - 1);
            uint32_t k = (uint32_t)floordiv2(y - x + n - 1);
            int ctx = 2 * colour + mod2(x);
            if (metropolis) ctx = 2 * ctx + (s == 12);
            uint32_t u = or_site_uniform(seed, r, k, t, (uint32_t)colour);
            T[i * M + j] = (u < thr[ctx]) ? 12 : 3;
        }
}

int64_t or_domino_observe(int n, const uint8_t *Tb, const uint8_t *Tw, uint32_t bin,
                          uint64_t *bin_sum)
{
    int W = 2 * n;
    uint8_t *faces = (uint8_t *)malloc((size_t)W * W);
    or_domino_to_faces(n, Tb, Tw, faces);
    int bx = (W + (int)bin - 1) / (int)bin;
    int64_t total = 0;
    for (int Y = 0; Y < W; ++Y)
        for (int X = 0; X < W; ++X) {
            uint8_t d = faces[Y * W + X];
            if (d == 2 || d == 3) {
                ++total;
                if (bin_sum) bin_sum[(Y / (int)bin) * bx + X / (int)bin] += 1;
            }
        }
    free(faces);
    return total;
}

int or_domino_sweeps(int n, uint8_t *Tb, uint8_t *Tw, const uint32_t *thr, int metropolis,
                     uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, or_obs *obs)
{
    for (uint32_t s = 0; s < nsweeps; ++s) {
        uint32_t t = t0 + s;
        for (uint32_t i = 0; i < 2; ++i) {
            /* the colour of the step and the sweep counter of its draws */
            uint32_t step = 2u * t + i;
            uint32_t colour = random_colours ? or_step_colour(seed, step, 2u) : i;
            uint32_t tc = random_colours ? step : t;
            if (colour == 0) {
                rotate(n, Tb, 0, thr, metropolis, seed, tc);
                update_white(n, Tw, Tb);
            } else {
                rotate(n, Tw, 1, thr, metropolis, seed, tc);
                update_black(n, Tb, Tw);
            }
        }
        if (obs && obs->obs_every && (t + 1) % obs->obs_every == 0) {
            int64_t v = or_domino_observe(n, Tb, Tw, obs->bin, obs->bin_sum);
            if (obs->scalar_sum) *obs->scalar_sum += v;
            if (obs->samples) *obs->samples += 1;
        }
    }
    return 0;
}
