/*
 * Serial CPU oracle for the parallel Glauber sweep of Keating & Sridhar,
 * "Random Tilings with the GPU" (arXiv:1804.07250).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no source with the HIP path: its own
 * Philox, its own domain builders, its own (unpacked) state representations.
 *
 * Representations (deliberately different from the GPU's bit-planes):
 *   domino      the paper's per-vertex tilestates split into the black and white
 *               arrays T_b and T_w, updated by the Rotate / Update steps of
 *               Section 2.2 (the bitwise Update formula is applied as printed);
 *   lozenge     a full int32 height H per triangular-lattice vertex;
 *   six-vertex  a full int32 height h per face (Figure "sixvertexh").
 *
 * Canonical exports (shared format, compared byte for byte):
 *   domino      uint8 per face of the 2n x 2n box, index Y*2n + X (Y = 0 is the
 *               southmost row), value = direction of the face's partner
 *               0:N 1:S 2:E 3:W, 0xFF outside the Aztec diamond;
 *   lozenge     int32 H per vertex of the sheared box (a+c+1) x (b+c+1), index
 *               Y*(a+c+1) + X, INT32_MIN outside the hexagon;
 *   six-vertex  int32 h per face of the (N+1) x (N+1) face box, index J*(N+1)+I.
 */
#ifndef TL_ORACLE_H
#define TL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 of Salmon, Moraes, Dror, Shaw (SC'11): out = f(ctr, key). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The 32-bit uniform of a site: bit (31-j) is bit (k & 31) of word (k>>5)&3 of
 * Philox(key = seed, ctr = (k>>7, r, t, 4j + c)), j = 0..31. */
uint32_t or_site_uniform(uint64_t seed, uint32_t r, uint32_t k, uint32_t t, uint32_t c);

/* Random colour order (the paper's RandomWalk): sweep t is the K colour steps
 * step = K t .. K t + K - 1, step `step` updating colour or_step_colour(seed,
 * step, K) with the site draws of sweep counter `step`.  The fixed order runs
 * colours 0 .. K-1 with sweep counter t. */
uint32_t or_step_colour(uint64_t seed, uint32_t step, uint32_t K);

/* Observable accumulator shared by the three models.  Cells are faces
 * (domino), vertices (lozenge) or vertices (six-vertex); bins are bin x bin
 * cells; bin_sum has bins_x*bins_y entries.  Any pointer may be NULL. */
typedef struct {
    uint32_t obs_every;   /* sample after sweep t when (t+1) % obs_every == 0; 0 = never */
    uint32_t bin;         /* bin edge in cells (>= 1) */
    uint64_t *bin_sum;    /* per-bin sums of the cell quantity over samples */
    int64_t *scalar_sum;  /* sum over samples of the whole-domain quantity */
    uint64_t *samples;    /* number of samples taken */
} or_obs;

/* Visit the sites of a colour class in reverse order (lozenge, six-vertex); a
 * proper colouring makes the result independent of this order. */
void or_set_reverse_order(int reverse);
extern int or_reverse_order;

/* ---------------- domino tilings of the Aztec diamond of order n --------- */
/* T_b and T_w each hold (2n+4) x (n+2) tilestates (see domino.c). */
int  or_domino_array_len(int n);
void or_domino_brick(int n, uint8_t *Tb, uint8_t *Tw);
int  or_domino_from_faces(int n, const uint8_t *faces, uint8_t *Tb, uint8_t *Tw, int allow_uncovered);
void or_domino_to_faces(int n, const uint8_t *Tb, const uint8_t *Tw, uint8_t *faces);
/* Tilestate s_v of box vertex (X, Y) (0 outside the box). */
int  or_domino_vertex_state(int n, const uint8_t *Tb, const uint8_t *Tw, int X, int Y);
/* Rotate the site at box vertex (X, Y) up (vertical pair) or down if it is
 * rotateable; returns 1 if the tiling changed. */
int  or_domino_flip(int n, uint8_t *Tb, uint8_t *Tw, int X, int Y, int up);
/* Run sweeps t0 .. t0+nsweeps-1.  thr has 4 entries (heat-bath, index
 * 2c + (x mod 2)) or 8 entries (lazy Metropolis, index 2*(2c + x mod 2) + cur). */
int  or_domino_sweeps(int n, uint8_t *Tb, uint8_t *Tw, const uint32_t *thr, int metropolis,
                      uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, or_obs *obs);
int64_t or_domino_observe(int n, const uint8_t *Tb, const uint8_t *Tw, uint32_t bin,
                          uint64_t *bin_sum);

/* ---------------- lozenge tilings of the a x b x c hexagon ---------------- */
int  or_lozenge_box(int a, int b, int c, int *W, int *H);
void or_lozenge_min(int a, int b, int c, int32_t *Hs);
void or_lozenge_max(int a, int b, int c, int32_t *Hs);
int  or_lozenge_flip(int a, int b, int c, int32_t *Hs, int X, int Y, int up);
/* thr: 1 entry (heat-bath) or 2 entries (Metropolis, index = current is up). */
int  or_lozenge_sweeps(int a, int b, int c, int32_t *Hs, const uint32_t *thr, int metropolis,
                       uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, or_obs *obs);
int64_t or_lozenge_observe(int a, int b, int c, const int32_t *Hs, uint32_t bin, uint64_t *bin_sum);

/* ---------------- six-vertex model, domain-wall boundary, N x N ----------- */
void or_sixv_min(int N, int32_t *h);
void or_sixv_max(int N, int32_t *h);
int  or_sixv_flip(int N, int32_t *h, int I, int J, int up);
/* thr: 16 entries (heat-bath, index = 4-bit mask of high diagonal faces
 * NE=1, NW=2, SW=4, SE=8) or 32 entries (Metropolis, index 2*mask + current is up). */
int  or_sixv_sweeps(int N, int32_t *h, const uint32_t *thr, int metropolis,
                    uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, or_obs *obs);
int64_t or_sixv_observe(int N, const int32_t *h, uint32_t bin, uint64_t *bin_sum);

/* ---------------- lozenge tilings of a general domain -------------------- */
/* w x h unit squares, heights on the (w+1) x (h+1) vertices (index Y*(w+1) + X),
 * site[Y*(w+1) + X] = 1 for vertices whose six triangles lie in the domain. */
int  or_lozr_flip(int W, int H, int32_t *Hs, const uint8_t *site, int X, int Y, int up);
int  or_lozr_sweeps(int W, int H, int32_t *Hs, const uint8_t *site, const uint32_t *thr, int metropolis,
                    uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours);

/* ---------------- six-vertex model on a general domain ------------------- */
/* W x H cell box, heights on its (W+1) x (H+1) points (index J*(W+1) + I),
 * site[J*(W+1) + I] = 1 for points whose four cells lie in the domain, 2 for
 * points on a free north edge (flips by thr_free, which may be NULL if there
 * are none). */
int  or_sixvr_flip(int W, int H, int32_t *h, const uint8_t *site, int side, int I, int J, int up);
int  or_sixvr_sweeps(int W, int H, int32_t *h, const uint8_t *site, const uint32_t *thr, const uint32_t *thr_free,
                     int metropolis, uint64_t seed, uint32_t t0, uint32_t nsweeps, int random_colours, int side,
                     int ox, int oy);

#ifdef __cplusplus
}
#endif
#endif
