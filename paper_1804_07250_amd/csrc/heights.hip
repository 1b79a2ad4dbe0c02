// Lozenge tilings of the a x b x c hexagon and the six-vertex model with
// domain-wall boundary: the two height-function models (Section 1.2).
//
// Both store one bit per height site (a 1-bit residual of the height):
//   lozenge    H(X, Y) mod 2 per triangular vertex; along (1,0), (0,1), (1,1) H
//              changes by 0 or -1, so the parity of two neighbours fixes their
//              difference.  Plane s = X mod 3 holds the vertices X = 3k + s of a
//              row, so one plane of a row is exactly one colour class (colour
//              (X + Y) mod 3).
//   six-vertex floor(h/2) mod 2 per face; neighbouring faces differ by +-1 and
//              h = (I + J) mod 2 + 2 floor(h/2), so the bit fixes the sign.
//              Plane p = I mod 2; colour (I mod 2) + 2 (J mod 2).
// A colour step updates one plane of every other row (six-vertex) or one plane
// of every row (lozenge); each site writes only its own bit, reading the other
// planes of its row and of the rows above and below.
//
// Lozenge move (Section 1.2, lozenge rotations): a vertex is rotateable iff its
// forward neighbours (X+1,Y), (X,Y+1), (X+1,Y+1) share a height f and its
// backward neighbours share f+1; up (add a cube) sets H = f+1, which has the
// parity of the backward neighbours, down sets H = f.
// Six-vertex move (c-flip): a face is flippable iff its four edge neighbours
// share a height m; up sets m+1.  A diagonal face is "high" iff it is at m+1.
// Context of the weights: sA = #high among NE, SW (corners carrying a) and
// sB = #high among NW, SE (corners carrying b); W_up/W_down depends on (sA, sB)
// only.
#include "../../include/tilings.h"
#include "height_common.hpp"
#include "internal.hpp"

namespace tl {

size_t height_words(HeightDev &d)
{
    if (d.model == TL_LOZENGE) {
        d.P = 3;
        d.rows = (uint32_t)(d.b + d.c + 1);
        d.K = (uint32_t)((d.a + d.c + 3) / 3);
    } else {
        d.P = 2;
        d.rows = (uint32_t)(d.N + 1);
        d.K = (uint32_t)((d.N + 2) / 2);
    }
    const uint32_t nw = (d.K + 31u) / 32u;
    d.ng = (nw + 3u) / 4u;
    d.RS = 4u * (d.ng + 2u);
    d.PS = (size_t)d.rows * d.RS;
    return d.P * d.PS;
}

namespace {

enum { kHeatBath = 0, kMetropolis = 1, kUniform = 2 };
static_assert(kHeatBath == kModeHeatBath && kMetropolis == kModeMetropolis && kUniform == kModeUniform,
              "kernel modes and TileJob modes agree");
// Tasks per work-group of a tile, and lanes per work-group of the multi-job
// kernels (512: room for the step kernels' registers when one-bit and
// bit-serial jobs share a launch); the tiled kernels take up to 1024 lanes
// (a quad of lanes per bit-serial task needs at most 69 registers per lane).
constexpr uint32_t kHeightThreads = 512;
constexpr uint32_t kTileThreads = 1024;
// Layout of a six-vertex threshold table (each layout is its own kernel
// instantiation, so its registers are allocated for it alone): 9 classes
// (sA, sB) [x2 for Metropolis], or 5 classes by sA + sB (heat-bath).  Lozenge
// tables always use kKindClass.
enum { kKindClass = 0, kKindSum = 1 };
static_assert(kKindClass == kTableClass && kKindSum == kTableSum, "table layouts agree");

// Instantiation KERNEL<mode, layout, flag> for a rule (mode), a table layout
// (kind) and a compile-time flag.
#define TL_HEIGHT_PICK_R(KERNEL, mode, kind, R)                                                 \
    ((mode) == kUniform ? KERNEL<kUniform, kKindClass, R>                                       \
     : (mode) == kMetropolis                                                                    \
         ? ((kind) == kKindSum ? KERNEL<kMetropolis, kKindSum, R> : KERNEL<kMetropolis, kKindClass, R>) \
     : (kind) == kKindSum ? KERNEL<kHeatBath, kKindSum, R> : KERNEL<kHeatBath, kKindClass, R>)
// And with two: the colour order (random) and site planes (masked domain).
#define TL_HEIGHT_PICK_RM(KERNEL, mode, kind, R, M)                                             \
    ((mode) == kUniform ? KERNEL<kUniform, kKindClass, R, M>                                    \
     : (mode) == kMetropolis                                                                    \
         ? ((kind) == kKindSum ? KERNEL<kMetropolis, kKindSum, R, M> : KERNEL<kMetropolis, kKindClass, R, M>) \
     : (kind) == kKindSum ? KERNEL<kHeatBath, kKindSum, R, M> : KERNEL<kHeatBath, kKindClass, R, M>)
#define TL_HEIGHT_PICK_ORDER_MASK(KERNEL, mode, kind, order, masked)                            \
    ((order) ? ((masked) ? TL_HEIGHT_PICK_RM(KERNEL, mode, kind, true, true)                    \
                         : TL_HEIGHT_PICK_RM(KERNEL, mode, kind, true, false))                  \
             : ((masked) ? TL_HEIGHT_PICK_RM(KERNEL, mode, kind, false, true)                   \
                         : TL_HEIGHT_PICK_RM(KERNEL, mode, kind, false, false)))

struct Geo {
    int model, a, b, c, N;
    const uint32_t *site;   // site planes of a masked domain (layout sPS, sRS), or nullptr
    size_t sPS;
    uint32_t sRS;
    const uint32_t *freep;  // six-vertex: planes of the free points (same layout), or nullptr
    int free_side;          // their side: 1 north, 2 south, 3 east, 4 west
};

__device__ __forceinline__ int imax(int p, int q) { return p > q ? p : q; }
__device__ __forceinline__ int imin(int p, int q) { return p < q ? p : q; }

// Lozenge: H_min / H_max at (X, Y) = (x + c, y + c).
__device__ __forceinline__ int loz_hmin(const Geo &g, int X, int Y) { return imax(0, imax(g.c - X, g.c - Y)); }
__device__ __forceinline__ int loz_hmax(const Geo &g, int X, int Y)
{
    return imin(g.c, imin(g.a + g.c - X, g.b + g.c - Y));
}
// Vertices of row Y inside the hexagon: X in [loz_xs, loz_xe].
__device__ __forceinline__ int loz_xs(const Geo &g, int Y) { return imax(0, Y - g.b); }
__device__ __forceinline__ int loz_xe(const Geo &g, int Y) { return imin(g.a + g.c, Y + g.a); }

__global__ void height_init_kernel(uint32_t *pa, uint32_t *pb, size_t PS, uint32_t RS, uint32_t rows, uint32_t P,
                                   Geo geo, int init_max)
{
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y, p = blockIdx.z;
    if (w >= RS || y >= rows || p >= P) return;
    uint32_t bits = 0u;
    if (w >= 4u) {
        const int dw = (int)w - 4;
        for (int bb = 0; bb < 32; ++bb) {
            const int k = dw * 32 + bb;
            if (geo.model == TL_LOZENGE) {
                const int X = 3 * k + (int)p, Y = (int)y;
                if (X > geo.a + geo.c || X < loz_xs(geo, Y) || X > loz_xe(geo, Y)) continue;
                const int H = init_max ? loz_hmax(geo, X, Y) : loz_hmin(geo, X, Y);
                bits |= (uint32_t)(H & 1) << bb;
            } else {
                const int I = 2 * k + (int)p, J = (int)y;
                if (I > geo.N) continue;
                const int h = init_max ? geo.N - abs(I + J - geo.N) : abs(I - J);
                bits |= (uint32_t)((h >> 1) & 1) << bb;
            }
        }
    }
    pa[p * PS + (size_t)y * RS + w] = bits;
    if (pb) pb[p * PS + (size_t)y * RS + w] = bits;
}

// Words of a group that one lane holds: all four when a lane has the task to
// itself (one-bit decisions), or word q alone when a quad of lanes shares it
// (lane q of the quad, bit-serial decisions).
template <uint32_t L>
constexpr int kWords = L == 4 ? 1 : 4;

template <int W>
__device__ __forceinline__ void hldw(const uint32_t *p, uint32_t q, uint32_t (&v)[W])
{
    if constexpr (W == 4)
        hld4(p, v);
    else
        v[0] = p[q];
}
template <int W>
__device__ __forceinline__ void hldw_plus1(const uint32_t *p, uint32_t q, uint32_t (&v)[W])
{
    if constexpr (W == 4)
        hld4_plus1(p, v);
    else
        v[0] = (p[q] >> 1) | (p[q + 1u] << 31);
}
template <int W>
__device__ __forceinline__ void hldw_minus1(const uint32_t *p, uint32_t q, uint32_t (&v)[W])
{
    if constexpr (W == 4)
        hld4_minus1(p, v);
    else
        v[0] = (p[q] << 1) | (p[(int)q - 1] >> 31);
}
template <int W>
__device__ __forceinline__ void hstw(uint32_t *p, uint32_t q, const uint32_t (&v)[W])
{
    if constexpr (W == 4)
        hst4(p, v);
    else
        p[q] = v[0];
}

// Bit-serial decisions of one group: plane by plane in one lane (L = 1,
// kPlanes generator calls per iteration), or by the quad of lanes that holds
// the group a word per lane (L = 4, this lane is q of the quad).
template <int NC, uint32_t L, uint32_t kPlanes = 1>
__device__ __forceinline__ void decide_sites(uint32_t k0, uint32_t k1, uint32_t g, uint32_t r, uint32_t t, uint32_t c,
                                             const uint32_t (&T)[NC], const uint32_t (&cm)[NC][kWords<L>],
                                             const uint32_t (&live)[kWords<L>], uint32_t q,
                                             uint32_t (&D)[kWords<L>])
{
    if constexpr (L == 4)
        decide32_quad<NC>(k0, k1, g, r, t, c, T, cm, live, q, D);
    else
        decide128<NC, kPlanes>(k0, k1, g, r, t, c, T, cm, live, D);
}

// Contexts: lozenge heat-bath 1, Metropolis 2 (current up); six-vertex
// heat-bath 9 classes 3*sA + sB, Metropolis 18 (2*class + current up), or,
// when a heat-bath table has 5 entries, classes by sA + sB alone.
template <int MODE, uint32_t L>
__device__ __forceinline__ void loz_decide(uint32_t k0, uint32_t k1, uint32_t g, uint32_t r, uint32_t t, uint32_t c,
                                           const Thr &Tall, const uint32_t (&R0)[4],
                                           const uint32_t (&cur)[kWords<L>], const uint32_t (&live)[kWords<L>],
                                           uint32_t q, uint32_t (&D)[kWords<L>])
{
    constexpr int W = kWords<L>;
    if constexpr (MODE == kUniform) {
#pragma unroll
        for (int w = 0; w < W; ++w) D[w] = ~R0[w];
    } else if constexpr (MODE == kHeatBath) {
        uint32_t T[1] = {Tall.v[0]}, cm[1][W];
#pragma unroll
        for (int w = 0; w < W; ++w) cm[0][w] = ~0u;
        decide_sites<1, L, 2>(k0, k1, g, r, t, c, T, cm, live, q, D);
    } else {
        uint32_t T[2] = {Tall.v[0], Tall.v[1]}, cm[2][W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            cm[0][w] = ~cur[w];
            cm[1][w] = cur[w];
        }
        decide_sites<2, L, 2>(k0, k1, g, r, t, c, T, cm, live, q, D);
    }
}

// Points of the free side (no neighbour across it): table Tall.v[kFreeBase ..]
// over the context (first diagonal at m+1) + 2 (second diagonal at m+1)
// [x2: current state up]; the diagonals (hSW, hSE here) are north SW, SE;
// south NW, NE; east SW, NW; west SE, NE.
template <int MODE, uint32_t L>
__device__ __forceinline__ void sixv_free_decide(uint32_t k0, uint32_t k1, uint32_t g, uint32_t r, uint32_t t,
                                                 uint32_t c, const Thr &Tall, const uint32_t (&R0)[4],
                                                 const uint32_t (&hSW)[kWords<L>], const uint32_t (&hSE)[kWords<L>],
                                                 const uint32_t (&cur)[kWords<L>], const uint32_t (&live)[kWords<L>],
                                                 uint32_t q, uint32_t (&D)[kWords<L>])
{
    constexpr int W = kWords<L>;
    if constexpr (MODE == kUniform) {
#pragma unroll
        for (int w = 0; w < W; ++w) D[w] = ~R0[w];
    } else {
        constexpr int NC = MODE == kMetropolis ? 8 : 4;
        uint32_t T[NC], cm[NC][W];
#pragma unroll
        for (int i = 0; i < NC; ++i) T[i] = Tall.v[Thr::kFreeBase + i];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const uint32_t m = ((x & 1) ? hSW[w] : ~hSW[w]) & ((x & 2) ? hSE[w] : ~hSE[w]);
                if (MODE == kMetropolis) {
                    cm[2 * x][w] = m & ~cur[w];
                    cm[2 * x + 1][w] = m & cur[w];
                } else {
                    cm[x][w] = m;
                }
            }
        decide_sites<NC, L>(k0, k1, g, r, t, c, T, cm, live, q, D);
    }
}

template <int MODE, int KIND, uint32_t L>
__device__ __forceinline__ void sixv_decide(uint32_t k0, uint32_t k1, uint32_t g, uint32_t r, uint32_t t, uint32_t c,
                                            const Thr &Tall, const uint32_t (&R0)[4], const uint32_t (&hNE)[kWords<L>],
                                            const uint32_t (&hNW)[kWords<L>], const uint32_t (&hSW)[kWords<L>],
                                            const uint32_t (&hSE)[kWords<L>], const uint32_t (&cur)[kWords<L>],
                                            const uint32_t (&live)[kWords<L>], uint32_t q, uint32_t (&D)[kWords<L>])
{
    constexpr int W = kWords<L>;
    if constexpr (MODE == kUniform) {
#pragma unroll
        for (int w = 0; w < W; ++w) D[w] = ~R0[w];
    } else if constexpr (KIND == kKindSum) {
        // thresholds that depend on sA + sB only (a = b): 5 classes s = 0..4
        // (Metropolis: x current state, down then up)
        constexpr int NC = MODE == kMetropolis ? 10 : 5;
        uint32_t T[NC], cm[NC][W];
#pragma unroll
        for (int i = 0; i < NC; ++i) T[i] = Tall.v[i];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t A0 = ~hNE[w] & ~hSW[w], A1 = hNE[w] ^ hSW[w], A2 = hNE[w] & hSW[w];
            const uint32_t B0 = ~hNW[w] & ~hSE[w], B1 = hNW[w] ^ hSE[w], B2 = hNW[w] & hSE[w];
            const uint32_t s[5] = {A0 & B0, (A0 & B1) | (A1 & B0), (A0 & B2) | (A1 & B1) | (A2 & B0),
                                   (A1 & B2) | (A2 & B1), A2 & B2};
#pragma unroll
            for (int x = 0; x < 5; ++x) {
                if constexpr (MODE == kMetropolis) {
                    cm[2 * x][w] = s[x] & ~cur[w];
                    cm[2 * x + 1][w] = s[x] & cur[w];
                } else {
                    cm[x][w] = s[x];
                }
            }
        }
        decide_sites<NC, L>(k0, k1, g, r, t, c, T, cm, live, q, D);
    } else {
        constexpr int NC = MODE == kMetropolis ? 18 : 9;
        uint32_t T[NC], cm[NC][W];
#pragma unroll
        for (int i = 0; i < NC; ++i) T[i] = Tall.v[i];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t A[3] = {~hNE[w] & ~hSW[w], hNE[w] ^ hSW[w], hNE[w] & hSW[w]};
            const uint32_t B[3] = {~hNW[w] & ~hSE[w], hNW[w] ^ hSE[w], hNW[w] & hSE[w]};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const uint32_t m = A[i] & B[j];
                    if (MODE == kMetropolis) {
                        cm[2 * (3 * i + j)][w] = m & ~cur[w];
                        cm[2 * (3 * i + j) + 1][w] = m & cur[w];
                    } else {
                        cm[3 * i + j][w] = m;
                    }
                }
        }
        decide_sites<NC, L>(k0, k1, g, r, t, c, T, cm, live, q, D);
    }
}

// Whether any lane of the quad has a nonzero value (the same answer in the
// four lanes, so that they call the shared decisions together).
template <uint32_t L>
__device__ __forceinline__ uint32_t group_any(uint32_t v)
{
    if constexpr (L == 4) return quad_or(v);
    return v;
}

// One lozenge group: sites k = 128 g + (0..127) of plane s0 in row Y.
// base(p, row) -> pointer to word 4 lg of that plane row (data words, pads
// around it).  lrow is the row index in the addressed array.
template <int MODE, bool MASKED, uint32_t L>
__device__ __forceinline__ void loz_group(uint32_t *base, size_t ps, uint32_t rs, uint32_t lrow, uint32_t lgrp,
                                          const Geo &geo, int Y, uint32_t g, uint32_t s0, uint32_t colour, uint32_t t,
                                          const Thr &Tall, uint32_t k0, uint32_t k1, uint32_t q)
{
    constexpr int W = kWords<L>;
    uint32_t R0[4] = {0u, 0u, 0u, 0u};
    if (MODE == kUniform) philox4x32_10(g, (uint32_t)Y, t, colour, k0, k1, R0);
    auto P = [&](uint32_t p, uint32_t r) { return base + p * ps + (size_t)r * rs + 4u + 4u * lgrp; };
    uint32_t O[W], f1[W], f2[W], f3[W], b1[W], b2[W], b3[W];
    hldw<W>(P(s0, lrow), q, O);
    hldw<W>(P(s0, lrow + 1), q, f2);
    hldw<W>(P(s0, lrow - 1), q, b2);
    if (s0 < 2) {
        hldw<W>(P(s0 + 1, lrow), q, f1);
        hldw<W>(P(s0 + 1, lrow + 1), q, f3);
    } else {
        hldw_plus1<W>(P(0, lrow), q, f1);
        hldw_plus1<W>(P(0, lrow + 1), q, f3);
    }
    if (s0 > 0) {
        hldw<W>(P(s0 - 1, lrow), q, b1);
        hldw<W>(P(s0 - 1, lrow - 1), q, b3);
    } else {
        hldw_minus1<W>(P(2, lrow), q, b1);
        hldw_minus1<W>(P(2, lrow - 1), q, b3);
    }
    // interior of row Y: X in (max(0, Y-b), min(a+c, Y+a)), X = 3k + s0
    const int xlo = imax(0, Y - geo.b), xhi = imin(geo.a + geo.c, Y + geo.a);
    const int klo = floordiv(xlo - (int)s0, 3) + 1, khi = floordiv(xhi - (int)s0 - 1, 3);
    // a masked domain: only its sites
    uint32_t sm[W];
#pragma unroll
    for (int w = 0; w < W; ++w) sm[w] = ~0u;
    if constexpr (MASKED) hldw<W>(geo.site + s0 * geo.sPS + (size_t)Y * geo.sRS + 4u + 4u * g, q, sm);
    uint32_t live[W], cur[W];
    uint32_t any = 0u;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int wi = W == 4 ? w : (int)q;   // the word's index in the group
        const uint32_t m = range_mask((int)(4 * g) + wi, klo, khi) & sm[w];
        live[w] = ~(f1[w] ^ f2[w]) & ~(f1[w] ^ f3[w]) & ~(b1[w] ^ b2[w]) & ~(b1[w] ^ b3[w]) & (f1[w] ^ b1[w]) & m;
        cur[w] = ~(O[w] ^ b1[w]);
        any |= live[w];
    }
    if (!group_any<L>(any)) return;
    uint32_t D[W];
    loz_decide<MODE, L>(k0, k1, g, (uint32_t)Y, t, colour, Tall, R0, cur, live, q, D);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t nw = (D[w] & b1[w]) | (~D[w] & f1[w]);
        O[w] = (O[w] & ~live[w]) | (nw & live[w]);
    }
    hstw<W>(P(s0, lrow), q, O);
}

// One six-vertex group: faces I = 2k + p, k = 128 g + (0..127), of row J.
template <int MODE, int KIND, bool MASKED, uint32_t L>
__device__ __forceinline__ void sixv_group(uint32_t *base, size_t ps, uint32_t rs, uint32_t lrow, uint32_t lgrp,
                                           const Geo &geo, int J, uint32_t g, uint32_t p, uint32_t colour, uint32_t t,
                                           const Thr &Tall, uint32_t k0, uint32_t k1, uint32_t q)
{
    constexpr int W = kWords<L>;
    uint32_t R0[4] = {0u, 0u, 0u, 0u};
    if (MODE == kUniform) philox4x32_10(g, (uint32_t)J, t, colour, k0, k1, R0);
    auto P = [&](uint32_t pl, uint32_t r) { return base + pl * ps + (size_t)r * rs + 4u + 4u * lgrp; };
    uint32_t O[W], Nn[W], Sn[W], E[W], Wn[W], NE[W], NW[W], SE[W], SW[W];
    hldw<W>(P(p, lrow), q, O);
    hldw<W>(P(p, lrow + 1), q, Nn);
    hldw<W>(P(p, lrow - 1), q, Sn);
    if (p == 0) {
        hldw<W>(P(1, lrow), q, E);
        hldw_minus1<W>(P(1, lrow), q, Wn);
        hldw<W>(P(1, lrow + 1), q, NE);
        hldw_minus1<W>(P(1, lrow + 1), q, NW);
        hldw<W>(P(1, lrow - 1), q, SE);
        hldw_minus1<W>(P(1, lrow - 1), q, SW);
    } else {
        hldw_plus1<W>(P(0, lrow), q, E);
        hldw<W>(P(0, lrow), q, Wn);
        hldw_plus1<W>(P(0, lrow + 1), q, NE);
        hldw<W>(P(0, lrow + 1), q, NW);
        hldw_plus1<W>(P(0, lrow - 1), q, SE);
        hldw<W>(P(0, lrow - 1), q, SW);
    }
    // interior faces 1 <= I <= N-1 (and, in a masked domain, its sites)
    const int klo = p == 0 ? 1 : 0, khi = (geo.N - 1 - (int)p) >> 1;
    uint32_t sm[W], fm[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        sm[w] = ~0u;
        fm[w] = 0u;
    }
    int side = 0;
    if constexpr (MASKED) {
        hldw<W>(geo.site + p * geo.sPS + (size_t)J * geo.sRS + 4u + 4u * g, q, sm);
        // points of the free side ignore their (absent) neighbour across it
        if (geo.freep) {
            hldw<W>(geo.freep + p * geo.sPS + (size_t)J * geo.sRS + 4u + 4u * g, q, fm);
            side = geo.free_side;
        }
    }
    const bool podd = ((p + (uint32_t)J) & 1u) != 0u;   // parity of I + J
    uint32_t live[W], up[W], hNE[W], hNW[W], hSW[W], hSE[W], cur[W];
    uint32_t any = 0u;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int wi = W == 4 ? w : (int)q;   // the word's index in the group
        const uint32_t m = range_mask((int)(4 * g) + wi, klo, khi) & sm[w];
        const uint32_t eEW = ~(E[w] ^ Wn[w]), eEN = ~(E[w] ^ Nn[w]), eES = ~(E[w] ^ Sn[w]);
        // free points: the three neighbours off the free side share m
        const uint32_t lf = side == 1   ? eEW & eES
                            : side == 2 ? eEW & eEN
                            : side == 3 ? ~(Wn[w] ^ Nn[w]) & ~(Wn[w] ^ Sn[w])
                            : side == 4 ? eEN & eES
                                        : 0u;
        live[w] = ((eEW & eEN & eES & ~fm[w]) | (lf & fm[w])) & m;
        // residual bit of m + 1 (m read off E, or W across a free east side)
        const uint32_t ref = side == 3 ? (E[w] & ~fm[w]) | (Wn[w] & fm[w]) : E[w];
        up[w] = podd ? ref : ~ref;
        hNE[w] = ~(NE[w] ^ up[w]);
        hNW[w] = ~(NW[w] ^ up[w]);
        hSW[w] = ~(SW[w] ^ up[w]);
        hSE[w] = ~(SE[w] ^ up[w]);
        cur[w] = ~(O[w] ^ up[w]);
        any |= live[w];
    }
    if (!group_any<L>(any)) return;
    uint32_t D[W];
    if constexpr (MASKED) {
        uint32_t li[W], lf[W], anyf = 0u;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            li[w] = live[w] & ~fm[w];
            lf[w] = live[w] & fm[w];
            anyf |= lf[w];
        }
        sixv_decide<MODE, KIND, L>(k0, k1, g, (uint32_t)J, t, colour, Tall, R0, hNE, hNW, hSW, hSE, cur, li, q, D);
        if (group_any<L>(anyf)) {
            uint32_t Df[W];
            // context diagonals beside the two cells the flip changes
            const uint32_t (&c0)[W] = side == 2 ? hNW : side == 4 ? hSE : hSW;
            const uint32_t (&c1)[W] = side == 1 ? hSE : side == 3 ? hNW : hNE;
            sixv_free_decide<MODE, L>(k0, k1, g, (uint32_t)J, t, colour, Tall, R0, c0, c1, cur, lf, q, Df);
#pragma unroll
            for (int w = 0; w < W; ++w) D[w] = (D[w] & ~fm[w]) | (Df[w] & fm[w]);
        }
    } else {
        sixv_decide<MODE, KIND, L>(k0, k1, g, (uint32_t)J, t, colour, Tall, R0, hNE, hNW, hSW, hSE, cur, live, q, D);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t nw = ~(D[w] ^ up[w]);
        O[w] = (O[w] & ~live[w]) | (nw & live[w]);
    }
    hstw<W>(P(p, lrow), q, O);
}

// Which plane of row y holds the sites of colour c (-1: none in this row).
__device__ __forceinline__ int colour_plane(const Geo &geo, int y, uint32_t c)
{
    if (geo.model == TL_LOZENGE) return (int)((c + 3u * 1024u - (uint32_t)y % 3u) % 3u);
    return ((c >> 1) == ((uint32_t)y & 1u)) ? (int)(c & 1u) : -1;
}

// Site rows: lozenge 1 .. b+c-1, six-vertex 1 .. N-1.
__device__ __forceinline__ bool site_row(const Geo &geo, int y, uint32_t rows)
{
    return y >= 1 && y <= (int)rows - 2;
}

// GEOM: the model when known at compile time (kGeomLozenge, kGeomSixv), or
// kGeomAny to read it from geo.
enum { kGeomAny = 0, kGeomLozenge = 1, kGeomSixv = 2 };
template <int MODE, int KIND, bool MASKED, uint32_t L = 1, int GEOM = kGeomAny>
__device__ __forceinline__ void height_group(uint32_t *base, size_t ps, uint32_t rs, uint32_t lrow, uint32_t lgrp,
                                             const Geo &geo, int y, uint32_t g, uint32_t colour, uint32_t t,
                                             const Thr &T, uint32_t k0, uint32_t k1, uint32_t q = 0)
{
    const int pl = colour_plane(geo, y, colour);
    if (pl < 0) return;
    if (GEOM == kGeomLozenge || (GEOM == kGeomAny && geo.model == TL_LOZENGE))
        loz_group<MODE, MASKED, L>(base, ps, rs, lrow, lgrp, geo, y, g, (uint32_t)pl, colour, t, T, k0, k1, q);
    else
        sixv_group<MODE, KIND, MASKED, L>(base, ps, rs, lrow, lgrp, geo, y, g, (uint32_t)pl, colour, t, T, k0, k1, q);
}

template <int MODE, int KIND, bool MASKED>
__global__ void __launch_bounds__(256) height_step_kernel(uint32_t *planes, size_t PS, uint32_t RS, uint32_t ng,
                                                          uint32_t rows, Geo geo, uint32_t colour, uint32_t t, Thr T,
                                                          uint32_t k0, uint32_t k1)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t g = gid % ng, y = gid / ng;
    if (!site_row(geo, (int)y, rows)) return;
    height_group<MODE, KIND, MASKED>(planes, PS, RS, y, g, geo, (int)y, g, colour, t, T, k0, k1);
}

// One tile of the multi-sweep kernel.  LDS: P planes x LR rows x LRS words,
// LRS = 4*(LG+2) (the pad groups hold the neighbouring groups, or zero).  Local
// row lr is global row R0 + lr, local group lg is global group G0 + lg.  With a
// row halo, the rows still valid before sweep s are [rps*s, LR - rps*s) (rps
// rows go stale per sweep on each side), and only those are computed.  Under
// the random colour order (RANDOM) step q of the launch (K per sweep) draws
// its colour and computes rows [q, LR - q).  Lozenge: every row holds sites
// of every colour; the block has a thread per (row, group) task (blockDim >=
// LR * LG) and thread tid handles group tid % LG of row base + tid / LG.
// Six-vertex: only rows of parity c >> 1 hold sites of colour c, so the
// threads cover those rows alone (blockDim >= ceil(LR / 2) * LG): thread tid
// handles group tid % LG of the (tid / LG)-th such row from base.
template <int MODE, int KIND, bool RANDOM, bool MASKED, int GEOM = kGeomAny>
__device__ __forceinline__ void height_tile(uint32_t *lds, const uint32_t *__restrict__ in,
                                            uint32_t *__restrict__ out, size_t PS, uint32_t RS, uint32_t ng,
                                            uint32_t rows, uint32_t P, const Geo &geo, uint32_t t0,
                                            uint32_t nsweeps, uint32_t TR, uint32_t TG, uint32_t HR, uint32_t HG,
                                            uint32_t tile_r, uint32_t tile_g, const Thr &T, uint32_t k0,
                                            uint32_t k1)
{
    const uint32_t LR = TR + 2 * HR, LG = TG + 2 * HG, LRS = 4 * (LG + 2);
    const uint32_t LPS = LR * LRS;
    const int R0 = (int)(tile_r * TR) - (int)HR, G0 = (int)(tile_g * TG) - (int)HG;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;

    // load LR rows x (LG + 2) groups (including the pad groups) per plane
    const uint32_t items = P * LR * (LG + 2);
    for (uint32_t i = tid; i < items; i += nt) {
        const uint32_t lg = i % (LG + 2), lr = (i / (LG + 2)) % LR, p = i / ((LG + 2) * LR);
        const int gr = R0 + (int)lr, gg = G0 - 1 + (int)lg;   // global group, -1 .. ng = pads
        uint32_t v[4] = {0u, 0u, 0u, 0u};
        if (gr >= 0 && gr < (int)rows && gg >= -1 && gg <= (int)ng)
            hld4(in + p * PS + (size_t)gr * RS + 4 + 4 * gg, v);
        hst4(lds + p * LPS + lr * LRS + 4 * lg, v);
    }
    __syncthreads();

    // Tasks: (row, group), six-vertex (row pair, group).  Bit-serial
    // decisions give each task a quad of lanes that spreads the planes over
    // its four lanes (L = 4), one-bit decisions one lane; a work-group with
    // fewer lanes than the tasks need takes them in turns.
    constexpr uint32_t L = MODE == kUniform ? 1u : 4u;
    const uint32_t ql = tid % L, slots = nt / L;
    const bool sixv = geo.model != TL_LOZENGE;
    const uint32_t ntasks = (sixv ? (LR + 1u) / 2u : LR) * LG;
    // (row, group) of this lane's first task, and the step to its next one,
    // divided once here rather than in every colour step
    const uint32_t task0 = tid / L, r00 = task0 / LG, lg00 = task0 % LG;
    const uint32_t step_r = slots / LG, step_g = slots % LG;
    const uint32_t K_colours = sixv ? 4u : 3u;
    const uint32_t rps = sixv ? 2u : 3u;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        for (uint32_t i = 0; i < K_colours; ++i) {
            // colour, sweep counter of the draws and valid rows of this step
            uint32_t c = i, t = t0 + s, base = HR ? rps * s : 0u, end = HR ? LR - rps * s : LR;
            if constexpr (RANDOM) {
                const uint32_t step = K_colours * t + i, q = K_colours * s + i;
                c = step_colour(step, K_colours, k0, k1);
                t = step;
                base = HR ? q : 0u;
                end = HR ? LR - q : LR;
            }
            uint32_t r0 = r00, lg = lg00;
            for (uint32_t task = task0; task < ntasks; task += slots) {
                const int gg = G0 + (int)lg;
                // six-vertex: the first row >= base of parity c >> 1, then every other row
                const uint32_t lr = sixv ? base + (((uint32_t)(R0 + (int)base) & 1u) ^ (c >> 1)) + 2u * r0 : base + r0;
                const int gr = R0 + (int)lr;
                if (gg >= 0 && gg < (int)ng && lr < end && lr >= 1 && lr + 1 < LR && site_row(geo, gr, rows))
                    height_group<MODE, KIND, MASKED, L, GEOM>(lds, LPS, LRS, lr, lg, geo, gr, (uint32_t)gg, c, t,
                                                              T, k0, k1, ql);
                // one-bit decisions: a lane per task, and every plan gives
                // the work-group at least as many lanes as tasks
                if constexpr (L == 1) break;
                r0 += step_r;
                lg += step_g;
                if (lg >= LG) {
                    lg -= LG;
                    ++r0;
                }
            }
            __syncthreads();
        }
    }

    const uint32_t oitems = P * TR * TG;
    for (uint32_t i = tid; i < oitems; i += nt) {
        const uint32_t ig = i % TG, ir = (i / TG) % TR, p = i / (TG * TR);
        const uint32_t orow = tile_r * TR + ir, og = tile_g * TG + ig;
        if (orow >= rows || og >= ng) continue;
        uint32_t v[4];
        hld4(lds + p * LPS + (ir + HR) * LRS + 4 * (ig + HG + 1), v);
        hst4(out + p * PS + (size_t)orow * RS + 4 + 4 * og, v);
    }
}

// Tiled multi-sweep kernels of one state: one work-group per tile.
template <int MODE, int KIND, bool RANDOM, bool MASKED>
__global__ void __launch_bounds__(kTileThreads) height_tiled_kernel(const uint32_t *__restrict__ in,
                                                            uint32_t *__restrict__ out, size_t PS, uint32_t RS,
                                                            uint32_t ng, uint32_t rows, uint32_t P, Geo geo,
                                                            uint32_t t0, uint32_t nsweeps, uint32_t TR, uint32_t TG,
                                                            uint32_t HR, uint32_t HG, uint32_t tiles_x, Thr T,
                                                            uint32_t k0, uint32_t k1)
{
    extern __shared__ uint32_t lds[];
    // plain work-group order: tiles of a hexagon differ in work, and the
    // round-robin dispatch over the XCDs balances them
    height_tile<MODE, KIND, RANDOM, MASKED, kGeomSixv>(lds, in, out, PS, RS, ng, rows, P, geo, t0, nsweeps, TR, TG,
                                                       HR, HG, blockIdx.x / tiles_x, blockIdx.x % tiles_x, T, k0, k1);
}
template <int MODE, int KIND, bool RANDOM, bool MASKED>
__global__ void __launch_bounds__(kTileThreads) loz_tiled_kernel(const uint32_t *__restrict__ in,
                                                        uint32_t *__restrict__ out, size_t PS, uint32_t RS,
                                                        uint32_t ng, uint32_t rows, uint32_t P, Geo geo, uint32_t t0,
                                                        uint32_t nsweeps, uint32_t TR, uint32_t TG, uint32_t HR,
                                                        uint32_t HG, uint32_t tiles_x, Thr T, uint32_t k0, uint32_t k1)
{
    extern __shared__ uint32_t lds[];
    height_tile<MODE, kKindClass, RANDOM, MASKED, kGeomLozenge>(lds, in, out, PS, RS, ng, rows, P, geo, t0, nsweeps,
                                                                TR, TG, HR, HG, blockIdx.x / tiles_x,
                                                                blockIdx.x % tiles_x, T, k0, k1);
}

// Multi-job kernel: work-group b runs tile items[b].tile of job items[b].job,
// with that job's geometry, plan, thresholds and key.
template <int MODE, int KIND, bool RANDOM, bool MASKED>
__device__ __forceinline__ void height_item(uint32_t *lds, const TileJob &j, uint32_t tile)
{
    const Geo geo{j.model, j.a, j.b, j.c, j.N, j.site, j.PS, j.RS, j.freep, j.free_side};
    height_tile<MODE, KIND, RANDOM, MASKED>(lds, j.in, j.out, j.PS, j.RS, j.ng, j.rows, j.P, geo, j.t0, j.S, j.TR,
                                            j.TG, j.HR,
                                    j.HG, tile / j.tiles_x, tile % j.tiles_x, j.T, j.key0, j.key1);
}

// Every job of a launch has the colour order RANDOM, and site planes iff MASKED.
template <int MODE, int KIND, bool RANDOM, bool MASKED>
__global__ void __launch_bounds__(kHeightThreads) height_items_kernel(const TileJob *__restrict__ jobs,
                                                                      const TileItem *__restrict__ items)
{
    extern __shared__ uint32_t lds[];
    const TileItem it = items[blockIdx.x];
    const TileJob &j = jobs[it.job];
    if constexpr (MODE == kHeatBath) {
        // one-bit jobs share the heat-bath launches (the lighter kernel body)
        if (j.mode == kUniform) {
            height_item<kUniform, kKindClass, RANDOM, MASKED>(lds, j, it.tile);
            return;
        }
    }
    height_item<MODE, KIND, RANDOM, MASKED>(lds, j, it.tile);
}

// The same with every rule and table layout in one launch: work-group b takes
// the kernel body of its job's rule and layout (the served ticks, where jobs of
// several rules share one launch instead of a launch per rule on streams
// joined by events).
template <bool RANDOM, bool MASKED>
__global__ void __launch_bounds__(kHeightThreads) height_items_mixed_kernel(const TileJob *__restrict__ jobs,
                                                                            const TileItem *__restrict__ items)
{
    extern __shared__ uint32_t lds[];
    const TileItem it = items[blockIdx.x];
    const TileJob &j = jobs[it.job];
    if (j.mode == kUniform)
        height_item<kUniform, kKindClass, RANDOM, MASKED>(lds, j, it.tile);
    else if (j.mode == kMetropolis)
        j.kind == kKindSum ? height_item<kMetropolis, kKindSum, RANDOM, MASKED>(lds, j, it.tile)
                           : height_item<kMetropolis, kKindClass, RANDOM, MASKED>(lds, j, it.tile);
    else
        j.kind == kKindSum ? height_item<kHeatBath, kKindSum, RANDOM, MASKED>(lds, j, it.tile)
                           : height_item<kHeatBath, kKindClass, RANDOM, MASKED>(lds, j, it.tile);
}

__device__ __forceinline__ uint32_t hbit(const uint32_t *pl, size_t PS, uint32_t RS, uint32_t p, uint32_t y,
                                         uint32_t k)
{
    return (pl[p * PS + (size_t)y * RS + 4 + (k >> 5)] >> (k & 31u)) & 1u;
}

// Bits k of a row word whose bit k is the point X0 + s k + p (the s planes
// of a row interleave their points) with u <= X0 + s k + p <= v.
__device__ __forceinline__ uint32_t word_mask(int X0, int p, int u, int v, int s)
{
    const int a = u - X0 - p, b = v - X0 - p;
    const int klo = a <= 0 ? 0 : (a + s - 1) / s, khi = b < 0 ? -1 : imin(31, b / s);
    if (klo > khi) return 0u;
    const uint32_t upto = khi >= 31 ? ~0u : (2u << khi) - 1u;
    return upto & ~((1u << klo) - 1u);
}

// Sum of the indices k of the set bits of x.
__device__ __forceinline__ uint32_t bit_index_sum(uint32_t x)
{
    return (uint32_t)__popc(x & 0xAAAAAAAAu) + 2u * (uint32_t)__popc(x & 0xCCCCCCCCu) +
           4u * (uint32_t)__popc(x & 0xF0F0F0F0u) + 8u * (uint32_t)__popc(x & 0xFF00FF00u) +
           16u * (uint32_t)__popc(x & 0xFFFF0000u);
}

// Heights of every point of a row, one wavefront per row.  A chunk is word m
// of each plane: lozenge vertices X in [96m, 96m + 96) (bit k of plane p is
// X = 96m + 3k + p), six-vertex faces I in [64m, 64m + 64) (I = 64m + 2k + p).
// Along a lozenge row H falls by one exactly where the residual bit differs
// from the previous vertex's.  Along a six-vertex row h moves by one at every
// face, and, the bit being bit 1 of h and h having the parity of I + J, it
// goes up exactly where the bit, the previous face's bit and that parity XOR
// to 1.  So each chunk's step words are XORs of its planes: phase one keeps
// them in LDS with the count of steps before the chunk (a wavefront prefix
// sum); phase two writes the row, consecutive lanes on consecutive points,
// each height the row's first one moved by popcounts of the steps up to it.
// LDS: nch words of counts, then 3 nch (lozenge) or 2 nch step words.
__global__ void __launch_bounds__(64) height_export_kernel(const uint32_t *pl, size_t PS, uint32_t RS, Geo geo,
                                                           uint32_t nch, int32_t *out)
{
    extern __shared__ uint32_t xl[];
    const int y = (int)blockIdx.x, lane = (int)threadIdx.x;
    const uint32_t *row = pl + (size_t)y * RS + 4;
    uint32_t *pre = xl, *steps = xl + nch;
    const bool loz = geo.model == TL_LOZENGE;
    const int P = loz ? 3 : 2, span = loz ? 96 : 64;
    // the row's points with a step, and (lozenge) its vertices
    const int xs = loz ? loz_xs(geo, y) : 0, xe = loz ? loz_xe(geo, y) : geo.N;
    int carry = 0;
    for (int m0 = 0; m0 < (int)nch; m0 += 64) {
        const int m = m0 + lane, X0 = span * m;
        const int lo = imax(xs, X0), hi = imin(xe, X0 + span - 1), L = imax(lo, xs + 1);
        uint32_t S[3] = {0u, 0u, 0u};
        int cnt = 0;
        if (m < (int)nch && lo <= hi) {
            if (loz) {
                const uint32_t W0 = row[m], W1 = row[PS + m], W2 = row[2 * PS + m];
                const uint32_t cin = X0 > xs ? row[2 * PS + m - 1] >> 31 : 0u;   // the vertex before X0
                S[0] = W0 ^ ((W2 << 1) | cin);
                S[1] = W1 ^ W0;
                S[2] = W2 ^ W1;
            } else {
                const uint32_t P0 = row[m], P1 = row[PS + m];
                const uint32_t cin = m > 0 ? row[PS + m - 1] >> 31 : 0u;   // the face before I = 64m
                const uint32_t par0 = (y & 1) ? ~0u : 0u;                  // parity of I + J, I even
                S[0] = P0 ^ ((P1 << 1) | cin) ^ par0;
                S[1] = P1 ^ P0 ^ ~par0;
            }
            for (int p = 0; p < P; ++p) cnt += __popc(S[p] & word_mask(X0, p, L, hi, P));
        }
        int incl = cnt;   // inclusive scan over the lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        if (m < (int)nch) {
            pre[m] = (uint32_t)(carry + incl - cnt);
            for (int p = 0; p < P; ++p) steps[P * m + p] = S[p];
        }
        carry += __shfl(incl, 63, 64);
    }
    __syncthreads();
    const int W = loz ? geo.a + geo.c + 1 : geo.N + 1;
    const int h0 = loz ? loz_hmin(geo, xs, y) : y;   // lozenge H at xs, six-vertex h(0, J) = J
    int32_t *o = out + (size_t)y * W;
    for (int X = lane; X < W; X += 64) {
        int32_t v = INT32_MIN;
        if (X >= xs && X <= xe) {
            const int m = X / span, X0 = span * m, L = imax(imax(xs, X0), xs + 1);
            int c = (int)pre[m];
            for (int p = 0; p < P; ++p) c += __popc(steps[P * m + p] & word_mask(X0, p, L, X, P));
            v = loz ? h0 - c : h0 + 2 * c - X;
        }
        o[X] = v;
    }
}

// Six-vertex observable: the type-c vertices (both diagonal pairs of faces
// around the vertex equal) counted into bins of B x B cells (cell (i-1, j-1) =
// vertex (i, j), 1 <= i, j <= N).  One thread per vertex row j and word w: the
// word holds vertices i = 2k+1 (faces I = 2k, 2k+1 from planes 0 and 1) and
// i = 2k+2 (faces 2k+1, 2k+2: plane 1 and plane 0 shifted by one site) for
// k = 32w .. 32w+31, so the test runs on whole words; the counts go to the
// bins by popcounts of the runs of cells that share a bin.
__global__ void sixv_observe_kernel(const uint32_t *pl, size_t PS, uint32_t RS, int N, uint32_t nw, uint32_t B,
                                    uint32_t bins_x, unsigned long long *bins)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t w = gid % nw, j = gid / nw + 1u;
    if (j > (uint32_t)N) return;
    const uint32_t *r0 = pl + (size_t)(j - 1) * RS + 4, *r1 = pl + (size_t)j * RS + 4;   // plane 0 rows
    const uint32_t *q0 = r0 + PS, *q1 = r1 + PS;                                          // plane 1 rows
    const uint32_t p0lo = r0[w], p0hi = r1[w], p1lo = q0[w], p1hi = q1[w];
    const uint32_t p0lo_s = (r0[w] >> 1) | (r0[w + 1] << 31), p0hi_s = (r1[w] >> 1) | (r1[w + 1] << 31);
    // i = 2k+1: a00 = p0[j-1][k], a11 = p1[j][k], a10 = p1[j-1][k], a01 = p0[j][k]
    uint32_t c_odd = ~(p0lo ^ p1hi) & ~(p1lo ^ p0hi);
    // i = 2k+2: a00 = p1[j-1][k], a11 = p0[j][k+1], a10 = p0[j-1][k+1], a01 = p1[j][k]
    uint32_t c_even = ~(p1lo ^ p0hi_s) & ~(p0lo_s ^ p1hi);
    c_odd &= range_mask((int)w, 0, (N - 1) / 2);
    c_even &= N >= 2 ? range_mask((int)w, 0, (N - 2) / 2) : 0u;
    // cells x = i - 1: x = 2k (odd i), x = 2k + 1 (even i), k = 32w + b
    const uint32_t by = (j - 1) / B, x_lo = 64u * w, x_hi = x_lo + 64u;
    for (uint32_t x = x_lo; x < x_hi;) {
        const uint32_t nxt = (x / B + 1u) * B < x_hi ? (x / B + 1u) * B : x_hi;
        // bits b with 2(32w + b) in [x, nxt) and 2(32w + b) + 1 in [x, nxt)
        const uint32_t e0 = (x - x_lo + 1u) / 2u, e1 = (nxt - x_lo + 1u) / 2u;   // even cells 2b in [x, nxt)
        const uint32_t o0 = (x - x_lo) / 2u, o1 = (nxt - x_lo) / 2u;             // odd cells 2b+1 in [x, nxt)
        auto bits = [](uint32_t lo, uint32_t hi) -> uint32_t {
            if (lo >= hi) return 0u;
            const uint32_t up = hi >= 32u ? ~0u : ((1u << hi) - 1u);
            return up & ~((1u << lo) - 1u);
        };
        const uint32_t cnt = (uint32_t)__popc(c_odd & bits(e0, e1)) + (uint32_t)__popc(c_even & bits(o0, o1));
        if (cnt) atomicAdd(&bins[(size_t)by * bins_x + x / B], (unsigned long long)cnt);
        x = nxt;
    }
}

// Six-vertex domain given by a mask: heights of the (h+1) x (w+1) points.  Off
// the domain INT32_MIN; boundary points take their fixed height; a site takes
// the value one away from a neighbour already known whose residual bit
// floor(h/2) mod 2 matches its own.  One thread per row J, walking east from
// each row segment's first point (fixed: it has a west side of a cell on the
// boundary), or, when the west side is free, one thread per column I walking
// north from each column segment's lowest point (fixed by its south side).
__global__ void sixv_region_export_kernel(const uint32_t *pl, size_t PS, uint32_t RS, const int32_t *anchor, int w,
                                          int h, int ox, int oy, int by_columns, int32_t *out)
{
    const int line = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (line > (by_columns ? w : h)) return;
    int32_t prev = 0;
    for (int step = 0; step <= (by_columns ? h : w); ++step) {
        const int I = by_columns ? line : step, J = by_columns ? step : line;
        const size_t v = (size_t)J * (w + 1) + I;
        const int32_t a = anchor[v];
        int32_t x = a;
        if (a == INT32_MAX) {
            // the state holds point (I, J) at (I + ox, J + oy) (even offsets)
            const uint32_t X = (uint32_t)(I + ox), Y = (uint32_t)(J + oy);
            const uint32_t bx = hbit(pl, PS, RS, X & 1u, Y, X >> 1);
            x = ((uint32_t)(((prev + 1) >> 1) & 1) == bx) ? prev + 1 : prev - 1;
        }
        out[v] = x;
        prev = x;
    }
}

// Lozenge domain given by a mask: heights of the (h+1) x (w+1) vertices, one
// thread per row Y.  Off the domain INT32_MIN; boundary vertices take their
// fixed height; a site is its west neighbour's height minus one where the
// parity bits differ (steps along (1,0) are 0 or -1).
__global__ void loz_region_export_kernel(const uint32_t *pl, size_t PS, uint32_t RS, const int32_t *anchor, int w,
                                         int h, int32_t *out)
{
    const int Y = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (Y > h) return;
    int32_t prev = 0;
    uint32_t pbit = 0u;
    for (int X = 0; X <= w; ++X) {
        const size_t v = (size_t)Y * (w + 1) + X;
        const int32_t a = anchor[v];
        const uint32_t bx = hbit(pl, PS, RS, (uint32_t)X % 3u, (uint32_t)Y, (uint32_t)X / 3u);
        const int32_t x = a == INT32_MAX ? prev - (int32_t)(bx ^ pbit) : a;
        out[v] = x;
        prev = x;
        pbit = bx;
    }
}

// Lozenge domain: H - H_min of every vertex of the domain into bins of B x B
// vertices, one thread per vertex.
__global__ void loz_region_volume_kernel(const int32_t *H, const int32_t *hmin, int w, int h, uint32_t B,
                                         uint32_t bins_x, unsigned long long *bins)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = (uint32_t)(w + 1) * (uint32_t)(h + 1);
    if (gid >= n) return;
    if (hmin[gid] == INT32_MIN) return;
    const int32_t q = H[gid] - hmin[gid];
    const uint32_t X = gid % (uint32_t)(w + 1), Y = gid / (uint32_t)(w + 1);
    if (q) atomicAdd(&bins[(size_t)(Y / B) * bins_x + X / B], (unsigned long long)q);
}

// Type-c cells of a masked six-vertex domain (both diagonal pairs of corner
// heights equal) into bins of B x B cells, one thread per cell.
__global__ void sixv_region_count_kernel(const int32_t *H, const uint8_t *cells, int w, int h, uint32_t B,
                                         uint32_t bins_x, unsigned long long *bins)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (uint32_t)w * (uint32_t)h) return;
    const int x = (int)(gid % (uint32_t)w), y = (int)(gid / (uint32_t)w);
    if (!cells[gid]) return;
    const size_t sw = (size_t)y * (w + 1) + x, nw = sw + (size_t)(w + 1);
    if (H[sw] == H[nw + 1] && H[sw + 1] == H[nw])
        atomicAdd(&bins[(size_t)((uint32_t)y / B) * bins_x + (uint32_t)x / B], 1ull);
}

// Lozenge observable: H - H_min per vertex, summed into bins of B x B cells.
// One wavefront per row Y, a lane per chunk X in [96m, 96m + 96): word m of
// the three planes holds the residual bits of those vertices (bit k of plane
// p is X = 96m + 3k + p).  H falls by one at every X > xs whose bit differs
// from the bit of X - 1, so XORs of the planes (plane 0 against plane 2
// shifted by one site) give the chunk's drops; a wavefront prefix sum of
// their counts gives every chunk its starting height.  Within a bin the sum
// of H over X in [u, v] is n H(u - 1) minus, for every drop d, the v - d + 1
// vertices from d on, and the sum of H_min = max(c - X, max(0, c - Y)) is an
// arithmetic series: popcounts and closed forms, no loop over vertices.
__global__ void __launch_bounds__(64) loz_observe_kernel(const uint32_t *pl, size_t PS, uint32_t RS, Geo geo,
                                                         uint32_t B, uint32_t bins_x, unsigned long long *bins)
{
    extern __shared__ unsigned long long rowbin[];
    const int Y = (int)blockIdx.x, lane = (int)threadIdx.x;
    for (uint32_t i = (uint32_t)lane; i < bins_x; i += 64u) rowbin[i] = 0ull;
    __syncthreads();
    const int xs = loz_xs(geo, Y), xe = loz_xe(geo, Y);
    const int h0 = imax(0, geo.c - Y), tc = geo.c - h0;   // H_min(X) = c - X for X < tc, else h0
    const uint32_t *row = pl + (size_t)Y * RS + 4;
    int carry = 0;   // drops in the chunks of earlier passes
    for (int m0 = xs / 96; m0 <= xe / 96; m0 += 64) {
        const int m = m0 + lane, X0 = 96 * m;
        const int lo = imax(xs, X0), hi = imin(xe, X0 + 95), L = imax(lo, xs + 1);
        uint32_t D[3] = {0u, 0u, 0u};
        int cnt = 0;
        if (lo <= hi) {
            const uint32_t W0 = row[m], W1 = row[PS + m], W2 = row[2 * PS + m];
            // the bit of X0 - 1 (plane 2, last bit of word m - 1), needed when X0 > xs
            const uint32_t cin = X0 > xs ? row[2 * PS + m - 1] >> 31 : 0u;
            D[0] = W0 ^ ((W2 << 1) | cin);
            D[1] = W1 ^ W0;
            D[2] = W2 ^ W1;
#pragma unroll
            for (int p = 0; p < 3; ++p) cnt += __popc(D[p] & word_mask(X0, p, L, hi, 3));
        }
        int incl = cnt;   // inclusive scan over the lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        const int total = __shfl(incl, 63, 64);
        if (lo <= hi) {
            int H = loz_hmin(geo, xs, Y) - carry - (incl - cnt);   // H before this chunk's drops
            for (int u = lo; u <= hi;) {
                const int j = u / (int)B, v = imin(hi, (j + 1) * (int)B - 1);
                const int du = imax(u, L);
                int c = 0;
                long long sd = 0;   // drops in [du, v] and the sum of their X
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    const uint32_t x = D[p] & word_mask(X0, p, du, v, 3);
                    const int cp = __popc(x);
                    c += cp;
                    sd += (long long)cp * (X0 + p) + 3ll * (long long)bit_index_sum(x);
                }
                const long long n = v - u + 1;
                const long long sumH = n * H - ((long long)c * (v + 1) - sd);
                long long sumMin = 0;
                const int aE = imin(v, tc - 1), bS = imax(u, tc);
                if (aE >= u) {
                    const long long na = aE - u + 1;
                    sumMin += na * geo.c - (long long)(u + aE) * na / 2;
                }
                if (bS <= v) sumMin += (long long)(v - bS + 1) * h0;
                if (sumH != sumMin) atomicAdd(&rowbin[j], (unsigned long long)(sumH - sumMin));
                H -= c;
                u = v + 1;
            }
        }
        carry += total;
    }
    __syncthreads();
    const size_t row_bins = (size_t)(Y / (int)B) * bins_x;
    for (uint32_t i = (uint32_t)lane; i < bins_x; i += 64u)
        if (rowbin[i]) atomicAdd(&bins[row_bins + i], rowbin[i]);
}

Geo geo_of(const HeightDev &d)
{
    return Geo{d.model, d.a, d.b, d.c, d.N, d.site, d.PS, d.RS, d.freep, d.free_side};
}

}  // namespace

hipError_t height_init(const HeightDev &d, int init_max, hipStream_t s)
{
    dim3 block(64), grid((d.RS + 63) / 64, d.rows, d.P);
    hipLaunchKernelGGL(height_init_kernel, grid, block, 0, s, d.planes, d.spare, d.PS, d.RS, d.rows, d.P, geo_of(d),
                       init_max);
    return hipGetLastError();
}

hipError_t height_colour_step(const HeightDev &d, int colour, uint32_t t, const Thr &T, int metropolis, uint64_t seed,
                              hipStream_t s, Timing *tm)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t threads = d.ng * d.rows;
    dim3 block(256), grid((threads + 255) / 256);
    const int mode = T.uniform() ? kUniform : (metropolis ? kMetropolis : kHeatBath);
    auto k = d.site ? TL_HEIGHT_PICK_R(height_step_kernel, mode, (int)table_kind(T), true)
                    : TL_HEIGHT_PICK_R(height_step_kernel, mode, (int)table_kind(T), false);
    return launch(tm, 1, k, grid, block, 0, s, d.planes, d.PS, d.RS, d.ng, d.rows, geo_of(d), (uint32_t)colour, t, T,
                  k0, k1);
}

HeightTile height_auto_tile(const HeightDev &d, bool uniform, bool metropolis)
{
    HeightTile t;
    if (d.rows <= 96 && d.ng <= 4) {   // whole domain in one tile, no halo
        t.TR = d.rows;
        t.TG = d.ng;
        t.S = 1u << 30;
        return t;
    }
    // Rows up to 8 groups wide are one tile wide (no column halo).  Bit-serial
    // decisions favour short tiles and few sweeps per launch, one-bit
    // decisions longer launches; measured on MI355X for the 1024 hexagon
    // (q = 1999/2000: 5 rows, 3 sweeps) and the N = 1024 squares (heat-bath
    // 4 rows and 6 sweeps, lazy Metropolis 8 and 8).
    t.TG = d.ng <= 8 ? d.ng : 4;
    if (uniform) {
        t.TR = 8;
        t.S = 16;
    } else if (d.model == TL_LOZENGE) {
        t.TR = 5;
        t.S = 3;
    } else {
        t.TR = metropolis ? 8 : 4;
        t.S = metropolis ? 8 : 6;
    }
    return t;
}

bool height_plan(const HeightDev &d, const HeightTile &tile, uint32_t S_max, TilePlan *p)
{
    if (d.rows == 0 || S_max == 0) return false;
    // halo rows invalidated per sweep, halo sites (per plane) per sweep; under
    // the random colour order each of the K steps may cost one of each
    const uint32_t K = d.model == TL_LOZENGE ? 3u : 4u;
    const uint32_t rows_per_sweep = tile.order ? K : (d.model == TL_LOZENGE ? 3u : 2u);
    const uint32_t cols_per_sweep = tile.order ? K : (d.model == TL_LOZENGE ? 1u : 2u);
    const uint32_t TG = tile.TG == 0 ? 1u : (tile.TG < d.ng ? tile.TG : d.ng);
    const uint32_t tiles_x = (d.ng + TG - 1) / TG;
    const uint32_t LG0 = TG + (tiles_x > 1 ? 2u : 0u);
    // six-vertex tiles run a thread per row pair (one row of each pair is idle
    // in every colour step), lozenge tiles a thread per row
    const uint32_t max_rows = (d.model == TL_LOZENGE ? 1u : 2u) * (kHeightThreads / LG0);
    if (max_rows < 2u * rows_per_sweep + 3u) return false;
    uint32_t TR = tile.TR == 0 ? 1u : (tile.TR < d.rows ? tile.TR : d.rows);
    if (TR < d.rows && TR > max_rows - 2u * rows_per_sweep) TR = max_rows - 2u * rows_per_sweep;
    if (TR >= d.rows && d.rows > max_rows) TR = max_rows - 2u * rows_per_sweep;
    const uint32_t tiles_y = (d.rows + TR - 1) / TR;
    uint32_t S = S_max < tile.S ? S_max : tile.S;
    if (tiles_x > 1 && S > 128u / cols_per_sweep) S = 128u / cols_per_sweep;
    if (tiles_y > 1 && S > (max_rows - TR) / (2u * rows_per_sweep)) S = (max_rows - TR) / (2u * rows_per_sweep);
    if (S == 0u) S = 1u;
    const uint32_t HR = tiles_y > 1 ? rows_per_sweep * S : 0u;
    const uint32_t HG = tiles_x > 1 ? 1u : 0u;
    const uint32_t LR = TR + 2 * HR, LG = TG + 2 * HG;
    const uint32_t tasks = height_task_rows(d.model, LR) * LG;
    const uint32_t lds = d.P * LR * 4u * (LG + 2u) * 4u;
    if (tasks > kHeightThreads || lds > 160u * 1024u) return false;
    p->S = S;
    p->TR = TR;
    p->TG = TG;
    p->HR = HR;
    p->HG = HG;
    p->tiles_x = tiles_x;
    p->tiles_y = tiles_y;
    // a thread per task, a quad per task for bit-serial decisions (the
    // kernel loops over the tasks when the work-group has fewer lanes)
    const uint32_t lanes = (tasks * (tile.lanes ? tile.lanes : 1u) + 63) / 64 * 64;
    const uint32_t cap = tile.items ? kHeightThreads : kTileThreads;
    p->threads = lanes < cap ? lanes : cap;
    p->lds = lds;
    p->order = tile.order;
    return true;
}

hipError_t height_tiled_sweeps(HeightDev &d, const HeightTile &tile, uint32_t t0, uint32_t nsw, const Thr &T,
                               int metropolis, uint64_t seed, hipStream_t s, Timing *tm)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t colours = d.model == TL_LOZENGE ? 3u : 4u;
    uint32_t done = 0;
    while (done < nsw) {
        TilePlan p;
        if (!height_plan(d, tile, nsw - done, &p)) return hipErrorInvalidConfiguration;
        const int mode = T.uniform() ? kUniform : (metropolis ? kMetropolis : kHeatBath);
#define TL_LOZ_PICK(R, M)                                                                              \
    (mode == kUniform ? loz_tiled_kernel<kUniform, kKindClass, R, M>                                   \
     : mode == kMetropolis ? loz_tiled_kernel<kMetropolis, kKindClass, R, M>                           \
                           : loz_tiled_kernel<kHeatBath, kKindClass, R, M>)
        const bool masked = d.site != nullptr;
        auto k = d.model == TL_LOZENGE
                     ? (p.order ? (masked ? TL_LOZ_PICK(true, true) : TL_LOZ_PICK(true, false))
                                : (masked ? TL_LOZ_PICK(false, true) : TL_LOZ_PICK(false, false)))
                     : TL_HEIGHT_PICK_ORDER_MASK(height_tiled_kernel, mode, (int)table_kind(T), p.order, masked);
#undef TL_LOZ_PICK
        hipError_t e = launch(tm, colours * p.S, k, dim3(p.tiles()), dim3(p.threads), p.lds, s,
                              (const uint32_t *)d.planes, d.spare, d.PS, d.RS, d.ng, d.rows, d.P, geo_of(d),
                              t0 + done, p.S, p.TR, p.TG, p.HR, p.HG, p.tiles_x, T, k0, k1);
        if (e != hipSuccess) return e;
        uint32_t *tmp = d.planes;
        d.planes = d.spare;
        d.spare = tmp;
        done += p.S;
    }
    return hipSuccess;
}

TileJob height_tile_job(const HeightDev &d, const TilePlan &p, uint32_t t0, const Thr &T, int metropolis,
                        uint64_t seed)
{
    TileJob j{};
    j.in = d.planes;
    j.out = d.spare;
    j.PS = d.PS;
    j.RS = d.RS;
    j.ng = d.ng;
    j.rows = d.rows;
    j.P = d.P;
    j.K = d.K;
    j.model = d.model;
    j.a = d.a;
    j.b = d.b;
    j.c = d.c;
    j.N = d.N;
    j.t0 = t0;
    j.S = p.S;
    j.TR = p.TR;
    j.TG = p.TG;
    j.HR = p.HR;
    j.HG = p.HG;
    j.tiles_x = p.tiles_x;
    j.order = p.order;
    j.mode = T.uniform() ? kModeUniform : (metropolis ? kModeMetropolis : kModeHeatBath);
    j.kind = T.uniform() ? (uint32_t)kTableClass : table_kind(T);
    j.site = d.site;
    j.freep = d.freep;
    j.free_side = d.free_side;
    j.key0 = (uint32_t)seed;
    j.key1 = (uint32_t)(seed >> 32);
    j.T = T;
    return j;
}

hipError_t height_items(const TileJob *jobs, const TileItem *items, uint32_t n_items, uint32_t threads, uint32_t lds,
                        uint32_t mode, uint32_t kind, uint32_t order, uint32_t masked, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (threads == 0 || threads > kHeightThreads || lds > 160u * 1024u || mode > 2u || kind > 1u)
        return hipErrorInvalidConfiguration;
    auto k = TL_HEIGHT_PICK_ORDER_MASK(height_items_kernel, (int)mode, (int)kind, order, masked);
    hipLaunchKernelGGL(k, dim3(n_items), dim3(threads), lds, s, jobs, items);
    return hipGetLastError();
}

hipError_t height_items_mixed(const TileJob *jobs, const TileItem *items, uint32_t n_items, uint32_t threads,
                              uint32_t lds, uint32_t order, uint32_t masked, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (threads == 0 || threads > kHeightThreads || lds > 160u * 1024u) return hipErrorInvalidConfiguration;
    auto k = order ? (masked ? height_items_mixed_kernel<true, true> : height_items_mixed_kernel<true, false>)
                   : (masked ? height_items_mixed_kernel<false, true> : height_items_mixed_kernel<false, false>);
    hipLaunchKernelGGL(k, dim3(n_items), dim3(threads), lds, s, jobs, items);
    return hipGetLastError();
}

hipError_t height_export(const HeightDev &d, int32_t *dev, hipStream_t s)
{
    // chunks of a row: 96 lozenge vertices or 64 six-vertex faces each
    const uint32_t nch = d.model == TL_LOZENGE ? (uint32_t)(d.a + d.c) / 96u + 1u : (uint32_t)d.N / 64u + 1u;
    const uint32_t shmem = 4u * nch * (d.model == TL_LOZENGE ? 4u : 3u);
    if (shmem > 64u * 1024u) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(height_export_kernel, dim3(d.rows), dim3(64), shmem, s, d.planes, d.PS, d.RS, geo_of(d), nch,
                       dev);
    return hipGetLastError();
}

hipError_t sixv_region_export(const HeightDev &d, const int32_t *anchor, int w, int h, int32_t *out, hipStream_t s)
{
    const int by_columns = d.free_side == 4 ? 1 : 0;
    const int lines = (by_columns ? w : h) + 1;
    hipLaunchKernelGGL(sixv_region_export_kernel, dim3((lines + 63) / 64), dim3(64), 0, s, d.planes, d.PS, d.RS,
                       anchor, w, h, d.ox, d.oy, by_columns, out);
    return hipGetLastError();
}

hipError_t loz_region_export(const HeightDev &d, const int32_t *anchor, int w, int h, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(loz_region_export_kernel, dim3((h + 64) / 64), dim3(64), 0, s, d.planes, d.PS, d.RS, anchor, w,
                       h, out);
    return hipGetLastError();
}

hipError_t loz_region_observe(const HeightDev &d, const int32_t *anchor, const int32_t *hmin, int w, int h,
                              int32_t *heights, uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s)
{
    hipError_t e = loz_region_export(d, anchor, w, h, heights, s);
    if (e != hipSuccess) return e;
    const uint32_t n = (uint32_t)(w + 1) * (uint32_t)(h + 1);
    hipLaunchKernelGGL(loz_region_volume_kernel, dim3((n + 255) / 256), dim3(256), 0, s, heights, hmin, w, h, B,
                       bins_x, bins);
    return hipGetLastError();
}

hipError_t sixv_region_observe(const HeightDev &d, const int32_t *anchor, const uint8_t *cells, int w, int h,
                               int32_t *heights, uint32_t B, uint32_t bins_x, unsigned long long *bins,
                               hipStream_t s)
{
    hipError_t e = sixv_region_export(d, anchor, w, h, heights, s);
    if (e != hipSuccess) return e;
    const uint32_t n = (uint32_t)w * (uint32_t)h;
    hipLaunchKernelGGL(sixv_region_count_kernel, dim3((n + 255) / 256), dim3(256), 0, s, heights, cells, w, h, B,
                       bins_x, bins);
    return hipGetLastError();
}

hipError_t height_observe(const HeightDev &d, uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s)
{
    if (d.model == TL_LOZENGE) {
        if ((size_t)bins_x * 8u > 64u * 1024u) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL(loz_observe_kernel, dim3(d.rows), dim3(64), bins_x * 8u, s, d.planes, d.PS, d.RS,
                           geo_of(d), B, bins_x, bins);
    } else {
        const uint32_t nw = 4u * d.ng, threads = nw * (uint32_t)d.N;
        hipLaunchKernelGGL(sixv_observe_kernel, dim3((threads + 255) / 256), dim3(256), 0, s, d.planes, d.PS, d.RS,
                           d.N, nw, B, bins_x, bins);
    }
    return hipGetLastError();
}

}  // namespace tl
