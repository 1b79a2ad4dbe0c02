// Domino tilings of the Aztec diamond: state initialisation, the colour-step
// kernels of the parallel Glauber sweep, the canonical export and the
// observable reduction.
//
// State (owner frame).  Every edge of the square lattice has exactly one
// endpoint of the owner colour omega = (n+1) mod 2; the owner sites of the
// order-n diamond form the grid (r, k) in [0,n)^2 with owner (r, k) at centred
// vertex (x, y) = (r-k, r+k+1-n).  Each owner keeps the crossing bits of its
// four edges in four bit-planes N, S, E, W (bit k of word k/32 of row r): the
// paper's tilestate s_v = N + 2S + 4E + 8W of Section 2.2, bit-sliced.  The
// other colour's site (r, k) sits at (r-k, r+k+2-n), directly north of owner
// (r, k); its edges are S = N(r,k), N = S(r+1,k+1), E = W(r+1,k), W = E(r,k+1).
//
// A colour step (Section 1.1.2, Section 2.2 "Rotate"): a site is rotateable iff
// N&S (two horizontal dominoes, tilestate 3) or E&W (two vertical dominoes,
// tilestate 12); it becomes vertical iff u < T[ctx] (the up-rotation) and
// horizontal otherwise; flipping toggles its four edge bits.  Owner steps touch
// only the owner's own bits; the other colour's step reads and writes bits of
// four owners, two of them shifted by one bit position.
//
// Two kernels run the same group update (128 sites of one row):
//   * a streaming kernel, one launch per colour step, on the state in HBM;
//   * a tiled kernel that loads a tile plus halo into LDS, runs S whole sweeps
//     there and writes the tile interior back (ping-pong buffers).  The halo is
//     recomputed redundantly with the same keyed draws, so results are
//     independent of the tiling.  In the owner frame one sweep invalidates one
//     row and one column of the halo on each side.
#include "device_common.hpp"
#include "internal.hpp"

namespace tl {

size_t domino_words(int n, uint32_t *ng, uint32_t *RS, size_t *PS)
{
    const uint32_t nw = (uint32_t)((n + 31) / 32);
    *ng = (nw + 3u) / 4u;
    *RS = 4u * (*ng + 1u);
    *PS = (size_t)(n + 1) * (*RS);
    return 4 * (*PS);
}

namespace {

// Faces of row y of the Aztec diamond are x in [-m, m-1], m = rows_half(n, y)
// (the same function gives the faces y in [-m, m-1] of column x).
__device__ __forceinline__ int rows_half(int n, int y) { return y >= 0 ? n - y : n + y + 1; }

// Is the segment between faces (x-1, y) and (x, y) of one row crossed by a
// domino of the brick tiling that covers the row from its west end?
__device__ __forceinline__ uint32_t brick_pair(int n, int x, int y)
{
    const int m = rows_half(n, y);
    return (m > 0 && x - 1 >= -m && x <= m - 1 && ((x - 1 + m) & 1) == 0) ? 1u : 0u;
}

// Writes the initial state into both buffers (a and, if non-null, b),
// including the zero padding.
__global__ void domino_init_kernel(uint32_t *a, uint32_t *b, size_t PS, uint32_t RS, int n, int init_max)
{
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = blockIdx.y;
    if (w >= RS || r > (uint32_t)n) return;
    uint32_t bits[4] = {0u, 0u, 0u, 0u};
    if (r < (uint32_t)n) {
        for (int bb = 0; bb < 32; ++bb) {
            const int k = (int)(w * 32u) + bb;
            if (k >= n) break;
            const int x = (int)r - k, y = (int)r + k + 1 - n;
            if (!init_max) {        // horizontal brick: N and S edges
                bits[0] |= brick_pair(n, x, y) << bb;
                bits[1] |= brick_pair(n, x, y - 1) << bb;
            } else {                // vertical brick (the transpose): E and W edges
                bits[2] |= brick_pair(n, y, x) << bb;
                bits[3] |= brick_pair(n, y, x - 1) << bb;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        a[p * PS + (size_t)r * RS + w] = bits[p];
        if (b) b[p * PS + (size_t)r * RS + w] = bits[p];
    }
}

__device__ __forceinline__ void ld4(const uint32_t *p, uint32_t (&v)[4])
{
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
}
__device__ __forceinline__ void st4(uint32_t *p, const uint32_t (&v)[4])
{
    *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
}

// Contexts of the domino tables: ctx = 2c + (x mod 2) (heat-bath) and
// 2(2c + x mod 2) + vertical (lazy Metropolis).  Sites (r, k) of both colours
// have x = r - k, so the x-parity alternates along the word.
template <bool METRO>
struct DomCtx;

template <>
struct DomCtx<false> {
    static constexpr int NC = 2;
    __device__ static void build(uint32_t r, uint32_t c, const Thr &Tall, const uint32_t (&)[4],
                                 uint32_t (&T)[2], uint32_t (&cm)[2][4])
    {
        const uint32_t even = (r & 1u) ? 0xAAAAAAAAu : 0x55555555u;  // sites with x even
        T[0] = Tall.v[2 * c];
        T[1] = Tall.v[2 * c + 1];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            cm[0][w] = even;
            cm[1][w] = ~even;
        }
    }
};

template <>
struct DomCtx<true> {
    static constexpr int NC = 4;
    __device__ static void build(uint32_t r, uint32_t c, const Thr &Tall, const uint32_t (&vert)[4],
                                 uint32_t (&T)[4], uint32_t (&cm)[4][4])
    {
        const uint32_t even = (r & 1u) ? 0xAAAAAAAAu : 0x55555555u;
#pragma unroll
        for (int i = 0; i < 4; ++i) T[i] = Tall.v[4 * c + i];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            cm[0][w] = even & ~vert[w];
            cm[1][w] = even & vert[w];
            cm[2][w] = ~even & ~vert[w];
            cm[3][w] = ~even & vert[w];
        }
    }
};

// Rule variants: general heat-bath, general lazy Metropolis, and uniform
// weights (every threshold 2^31: a site goes up iff the top bit of its uniform
// is 0, so one Philox call decides all 128 sites and does not depend on the
// state; it is issued first to overlap the memory latency).
enum { kHeatBath = 0, kMetropolis = 1, kUniform = 2 };
static_assert(kHeatBath == kModeHeatBath && kMetropolis == kModeMetropolis && kUniform == kModeUniform,
              "kernel modes and TileJob modes agree");

// Are all thresholds of colour c 2^31 (ratio 1, as in the first colour of
// two-periodic weights)?  Then the top bit of each site's uniform decides it
// alone, and plane 0 settles every site of the group.
template <int MODE>
__device__ __forceinline__ bool one_bit_colour(const Thr &Tall, uint32_t c)
{
    constexpr uint32_t NC = MODE == kMetropolis ? 4u : 2u;
    bool all = true;
#pragma unroll
    for (uint32_t i = 0; i < NC; ++i) all = all && Tall.v[NC * c + i] == 0x80000000u;
    return all;
}

template <int MODE>
__device__ __forceinline__ void decide_group(uint32_t key0, uint32_t key1, uint32_t g, uint32_t r, uint32_t t,
                                             uint32_t c, const Thr &Tall, const uint32_t (&R0)[4],
                                             const uint32_t (&vert)[4], const uint32_t (&live)[4], uint32_t (&D)[4])
{
    if (MODE == kUniform) {
#pragma unroll
        for (int w = 0; w < 4; ++w) D[w] = ~R0[w];
    } else if (one_bit_colour<MODE>(Tall, c)) {
        // the draw of plane 0, as the bit-serial comparison makes it first
        uint32_t R[4];
        philox4x32_10(g, r, t, c, key0, key1, R);
#pragma unroll
        for (int w = 0; w < 4; ++w) D[w] = ~R[w];
    } else {
        constexpr int NC = DomCtx<MODE == kMetropolis>::NC;
        uint32_t T[NC], cm[NC][4];
        DomCtx<MODE == kMetropolis>::build(r, c, Tall, vert, T, cm);
        decide128<NC>(key0, key1, g, r, t, c, T, cm, live, D);
    }
}

// Owner colour step on the 128 owner sites of group g of row r.  pN..pW point at
// word 4g of row r in the four planes (global memory or LDS).
template <int MODE>
__device__ __forceinline__ void owner_group(uint32_t *pN, uint32_t *pS, uint32_t *pE, uint32_t *pW, uint32_t r,
                                            uint32_t g, uint32_t c, uint32_t t, const Thr &Tall, uint32_t key0,
                                            uint32_t key1)
{
    uint32_t R0[4] = {0u, 0u, 0u, 0u};
    if (MODE == kUniform) philox4x32_10(g, r, t, c, key0, key1, R0);
    uint32_t N[4], S[4], E[4], W[4];
    ld4(pN, N);
    ld4(pS, S);
    ld4(pE, E);
    ld4(pW, W);
    uint32_t horiz[4], vert[4], live[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        horiz[w] = N[w] & S[w];
        vert[w] = E[w] & W[w];
        live[w] = horiz[w] | vert[w];
    }
    if ((live[0] | live[1] | live[2] | live[3]) == 0u) return;
    uint32_t D[4];
    decide_group<MODE>(key0, key1, g, r, t, c, Tall, R0, vert, live, D);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t F = (horiz[w] & D[w]) | (vert[w] & ~D[w]);
        N[w] ^= F;
        S[w] ^= F;
        E[w] ^= F;
        W[w] ^= F;
    }
    st4(pN, N);
    st4(pS, S);
    st4(pE, E);
    st4(pW, W);
}

// Other-colour step on the 128 sites of group g of row r.  rowN, rowE point at
// word 4g of owner row r (planes N, E); rowS1, rowW1 at word 4g of owner row r+1
// (planes S, W).  Word 4g+4 of rowE and rowS1 must exist (padding).  Bit 0 of
// the first word of a group in the shifted planes belongs to the previous
// group's last site, so the first and the carry words are updated atomically.
template <int MODE>
__device__ __forceinline__ void other_group(uint32_t *rowN, uint32_t *rowE, uint32_t *rowS1, uint32_t *rowW1,
                                            uint32_t r, uint32_t g, uint32_t c, uint32_t t, const Thr &Tall,
                                            uint32_t key0, uint32_t key1, bool has_next = true)
{
    // has_next = false: the group is the last of its row and the row has no pad
    // group after it (compact LDS rows); its word 4 reads as zero and its carry
    // bit (site k = 128 g + 127 >= n - 1, never a site of this colour) is zero.
    uint32_t R0[4] = {0u, 0u, 0u, 0u};
    if (MODE == kUniform) philox4x32_10(g, r, t, c, key0, key1, R0);
    uint32_t oN[4], oE[4], oS1[4], oW1[4];
    ld4(rowN, oN);
    ld4(rowE, oE);
    ld4(rowS1, oS1);
    ld4(rowW1, oW1);
    const uint32_t eNext = has_next ? rowE[4] : 0u, sNext = has_next ? rowS1[4] : 0u;
    uint32_t horiz[4], vert[4], live[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t eHi = (w < 3) ? oE[w + 1] : eNext;
        const uint32_t sHi = (w < 3) ? oS1[w + 1] : sNext;
        const uint32_t sS = oN[w], sE = oW1[w];
        const uint32_t sN = (oS1[w] >> 1) | (sHi << 31);
        const uint32_t sW = (oE[w] >> 1) | (eHi << 31);
        horiz[w] = sN & sS;
        vert[w] = sE & sW;
        live[w] = horiz[w] | vert[w];
    }
    if ((live[0] | live[1] | live[2] | live[3]) == 0u) return;
    uint32_t D[4];
    decide_group<MODE>(key0, key1, g, r, t, c, Tall, R0, vert, live, D);
    uint32_t F[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        F[w] = (horiz[w] & D[w]) | (vert[w] & ~D[w]);
        oN[w] ^= F[w];
        oW1[w] ^= F[w];
    }
    st4(rowN, oN);
    st4(rowW1, oW1);
    // shifted planes: bit k+1 <- F bit k
    atomicXor(&rowE[0], F[0] << 1);
    atomicXor(&rowS1[0], F[0] << 1);
#pragma unroll
    for (int w = 1; w < 4; ++w) {
        const uint32_t m = (F[w] << 1) | (F[w - 1] >> 31);
        rowE[w] = oE[w] ^ m;
        rowS1[w] = oS1[w] ^ m;
    }
    if (has_next && (F[3] >> 31)) {
        atomicXor(&rowE[4], 1u);
        atomicXor(&rowS1[4], 1u);
    }
}

// ---------------------------------------------------------- streaming kernels
template <int MODE>
__global__ void __launch_bounds__(256) domino_owner_step(uint32_t *planes, size_t PS, uint32_t RS, uint32_t ng,
                                                         uint32_t n, uint32_t c, uint32_t t, Thr Tall,
                                                         uint32_t key0, uint32_t key1)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t g = gid % ng, r = gid / ng;
    if (r >= n) return;
    uint32_t *base = planes + (size_t)r * RS + 4u * g;
    owner_group<MODE>(base, base + PS, base + 2 * PS, base + 3 * PS, r, g, c, t, Tall, key0, key1);
}

template <int MODE>
__global__ void __launch_bounds__(256) domino_other_step(uint32_t *planes, size_t PS, uint32_t RS, uint32_t ng,
                                                         uint32_t n, uint32_t c, uint32_t t, Thr Tall,
                                                         uint32_t key0, uint32_t key1)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t g = gid % ng, r = gid / ng;
    if (r + 1u >= n) return;   // the other colour has rows 0 .. n-2
    uint32_t *row = planes + (size_t)r * RS + 4u * g;
    other_group<MODE>(row, row + 2 * PS, row + PS + RS, row + 3 * PS + RS, r, g, c, t, Tall, key0, key1);
}

// -------------------------------------------------------------- tiled kernel
// Block = one tile.  Local (lr, lg) is global row R0 + lr, group G0 + lg.  LDS:
// 4 planes x LR rows x LRS words (LRS = domino_lds_row_words(LG): the LG groups, the neighbouring group
// the shifted planes read, and an odd slot count).
// One thread per (row, group) task; blockDim >= LR * LG.
// One tile of the multi-sweep kernel: TR owner rows x TG groups (tile index
// (tile_r, tile_g)) plus HR halo rows and HG halo groups on each side are
// loaded into LDS, advanced nsweeps sweeps there, and the interior written to
// `out`.  Halo cells repeat their neighbours' keyed draws, so the interior
// matches the sweep of the whole state; halo rows go stale one per sweep from
// each side, so sweep s computes only rows [s, LR - s).  Under the random
// colour order (RANDOM) step q of the launch (2 per sweep) draws its colour
// and computes rows [q, LR - q), the halo covering 2 rows per sweep.  The block
// has a thread per (row, group) task (blockDim >= LR * LG, as every launch
// plan gives): thread tid handles group tid / LR of row base + tid % LR, so
// the 16 lanes an LDS access serves at once are 16 rows of one group, which
// the odd row stride spreads over distinct banks.
template <int MODE, bool RANDOM>
__device__ __forceinline__ void domino_tile(uint32_t *lds, const uint32_t *__restrict__ in,
                                            uint32_t *__restrict__ out, size_t PS, uint32_t RS, uint32_t ng,
                                            uint32_t n, uint32_t omega, uint32_t t0, uint32_t nsweeps, uint32_t TR,
                                            uint32_t TG, uint32_t HR, uint32_t HG, uint32_t tile_r, uint32_t tile_g,
                                            const Thr &Tall, uint32_t key0, uint32_t key1)
{
    const uint32_t LR = TR + 2 * HR, LG = TG + 2 * HG, LRS = domino_lds_row_words(LG);
    const uint32_t LPS = LR * LRS;
    const int R0 = (int)(tile_r * TR) - (int)HR, G0 = (int)(tile_g * TG) - (int)HG;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;

    // load tile + halo (zero outside the state), one uint4 per item
    const uint32_t items = 4 * LR * (LG + 1);
    for (uint32_t i = tid; i < items; i += nt) {
        const uint32_t lg = i % (LG + 1), lr = (i / (LG + 1)) % LR, p = i / ((LG + 1) * LR);
        const int gr = R0 + (int)lr, gg = G0 + (int)lg;
        uint32_t v[4] = {0u, 0u, 0u, 0u};
        if (lg < LG && gr >= 0 && gr < (int)n && gg >= 0 && gg < (int)ng)
            ld4(in + p * PS + (size_t)gr * RS + 4 * gg, v);
        st4(lds + p * LPS + lr * LRS + 4 * lg, v);
    }
    __syncthreads();

    const uint32_t r0 = tid % LR, lg = tid / LR;
    const int gg = G0 + (int)lg;
    const bool lane = lg < LG && gg >= 0 && gg < (int)ng;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        for (uint32_t i = 0; i < 2; ++i) {
            // colour, sweep counter of the draws and valid rows of this step
            uint32_t c = i, t = t0 + s, base = HR ? s : 0u, end = HR ? LR - s : LR;
            if constexpr (RANDOM) {
                const uint32_t step = 2u * t + i, q = 2u * s + i;
                c = step_colour(step, 2u, key0, key1);
                t = step;
                base = HR ? q : 0u;
                end = HR ? LR - q : LR;
            }
            const uint32_t lr = base + r0;
            const int gr = R0 + (int)lr;
            if (lane && lr < end && gr >= 0 && gr < (int)n) {
                uint32_t *pN = lds + lr * LRS + 4 * lg;
                if (c == omega)
                    owner_group<MODE>(pN, pN + LPS, pN + 2 * LPS, pN + 3 * LPS, (uint32_t)gr, (uint32_t)gg, c, t,
                                      Tall, key0, key1);
                else if (lr + 1 < LR)
                    other_group<MODE>(pN, pN + 2 * LPS, pN + LPS + LRS, pN + 3 * LPS + LRS, (uint32_t)gr,
                                      (uint32_t)gg, c, t, Tall, key0, key1);
            }
            __syncthreads();
        }
    }

    // store the interior
    const uint32_t oitems = 4 * TR * TG;
    for (uint32_t i = tid; i < oitems; i += nt) {
        const uint32_t ig = i % TG, ir = (i / TG) % TR, p = i / (TG * TR);
        const uint32_t orow = tile_r * TR + ir, og = tile_g * TG + ig;
        if (orow >= n || og >= ng) continue;
        uint32_t v[4];
        ld4(lds + p * LPS + (ir + HR) * LRS + 4 * (ig + HG), v);
        st4(out + p * PS + (size_t)orow * RS + 4 * og, v);
    }
}

// Tiled multi-sweep kernel of one state: one work-group per tile.
template <int MODE, bool RANDOM>
__global__ void __launch_bounds__(1024) domino_tiled_kernel(const uint32_t *__restrict__ in,
                                                            uint32_t *__restrict__ out, size_t PS, uint32_t RS,
                                                            uint32_t ng, uint32_t n, uint32_t omega, uint32_t t0,
                                                            uint32_t nsweeps, uint32_t TR, uint32_t TG,
                                                            uint32_t HR, uint32_t HG, uint32_t tiles_x,
                                                            Thr Tall, uint32_t key0, uint32_t key1)
{
    extern __shared__ uint32_t lds[];
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    domino_tile<MODE, RANDOM>(lds, in, out, PS, RS, ng, n, omega, t0, nsweeps, TR, TG, HR, HG, tile / tiles_x,
                              tile % tiles_x, Tall, key0, key1);
}

// ------------------------------------------------ register-resident tiles
// The tiles, halo and draws of domino_tile with the state held in registers:
// wavefront w of the block holds local group w (LG wavefronts), lane l local
// row l (LR <= 64), sixteen words per lane (the group's four words in each of
// the four planes).  An owner step touches only a lane's own words.  The other
// colour's site (r, k) reads owner row r + 1, which is the next lane (a DPP
// wavefront shift), and bit 0 of the next group's first E word (row r) and S
// word (row r + 1), which live in the next wavefront and are exchanged through
// LDS; its flips change row r + 1's S and W planes (shifted back to the next
// lane) and, through the carry of the group's last site, bit 0 of those two
// words of the next group (LDS again).  The rows computed in each step, and
// every value written, are those of domino_tile.
constexpr uint32_t kRegRows = 64, kRegGroups = 16;

// Lane l receives lane l+1's value (lane_next) or lane l-1's (lane_prev);
// the lane past either end of the wavefront receives 0.
__device__ __forceinline__ uint32_t lane_next(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, true);   // wave_shl:1
}
__device__ __forceinline__ uint32_t lane_prev(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, true);   // wave_shr:1
}

template <int MODE, bool RANDOM>
__global__ void __launch_bounds__(1024) domino_reg_kernel(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                          size_t PS, uint32_t RS, uint32_t ng, uint32_t n,
                                                          uint32_t omega, uint32_t t0, uint32_t nsweeps, uint32_t TR,
                                                          uint32_t TG, uint32_t HR, uint32_t HG, uint32_t tiles_x,
                                                          Thr Tall, uint32_t key0, uint32_t key1)
{
    // First words of E and S published for the previous group, and either the
    // carries (bit-serial decisions: a second barrier) or, for one-bit
    // decisions, the bits of the group's last site from which the next group
    // computes that carry itself (one barrier per other-colour step; the
    // arrays alternate between consecutive such steps, so a wavefront that
    // runs ahead never overwrites what a slower one has still to read).
    constexpr bool kOneBarrier = MODE == kUniform;
    __shared__ uint32_t xE[2][kRegGroups][kRegRows], xS[2][kRegGroups][kRegRows], xC[2][kRegGroups][kRegRows];
    uint32_t xb = 0;   // buffer of the next other-colour step
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t tile_r = tile / tiles_x, tile_g = tile % tiles_x;
    const uint32_t LR = TR + 2 * HR, LG = TG + 2 * HG;
    const int R0 = (int)(tile_r * TR) - (int)HR, G0 = (int)(tile_g * TG) - (int)HG;
    const uint32_t lr = threadIdx.x & (kRegRows - 1u), lg = threadIdx.x / kRegRows;
    const int gr = R0 + (int)lr, gg = G0 + (int)lg;
    const bool mine = lr < LR && gr >= 0 && gr < (int)n && gg >= 0 && gg < (int)ng;
    uint32_t N[4] = {0u, 0u, 0u, 0u}, S[4] = {0u, 0u, 0u, 0u}, E[4] = {0u, 0u, 0u, 0u}, W[4] = {0u, 0u, 0u, 0u};
    if (mine) {
        const uint32_t *p = in + (size_t)gr * RS + 4 * gg;
        ld4(p, N);
        ld4(p + PS, S);
        ld4(p + 2 * PS, E);
        ld4(p + 3 * PS, W);
    }
    const bool has_next = lg + 1u < LG;
    for (uint32_t s = 0; s < nsweeps; ++s) {
        for (uint32_t i = 0; i < 2; ++i) {
            uint32_t c = i, t = t0 + s, base = HR ? s : 0u, end = HR ? LR - s : LR;
            if constexpr (RANDOM) {
                const uint32_t step = 2u * t + i, q = 2u * s + i;
                c = step_colour(step, 2u, key0, key1);
                t = step;
                base = HR ? q : 0u;
                end = HR ? LR - q : LR;
            }
            const bool act = mine && lr >= base && lr < end;
            uint32_t R0v[4] = {0u, 0u, 0u, 0u};
            if (MODE == kUniform) philox4x32_10((uint32_t)gg, (uint32_t)gr, t, c, key0, key1, R0v);
            if (c == omega) {
                uint32_t horiz[4], vert[4], live[4], any = 0u;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    horiz[w] = N[w] & S[w];
                    vert[w] = E[w] & W[w];
                    live[w] = horiz[w] | vert[w];
                    any |= live[w];
                }
                if (act && any) {
                    uint32_t D[4];
                    decide_group<MODE>(key0, key1, (uint32_t)gg, (uint32_t)gr, t, c, Tall, R0v, vert, live, D);
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const uint32_t F = (horiz[w] & D[w]) | (vert[w] & ~D[w]);
                        N[w] ^= F;
                        S[w] ^= F;
                        E[w] ^= F;
                        W[w] ^= F;
                    }
                }
            } else {
                uint32_t S1[4], W1[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    S1[w] = lane_next(S[w]);
                    W1[w] = lane_next(W[w]);
                }
                xE[xb][lg][lr] = E[0];
                xS[xb][lg][lr] = S[0];
                if constexpr (kOneBarrier) {
                    // the last site (127) of this group: its N bit, the W bit of
                    // the row above, its decision, and whether it may flip
                    const uint32_t may = act && lr + 1u < LR ? 8u : 0u;
                    xC[xb][lg][lr] = (N[3] >> 31) | ((W1[3] >> 31) << 1) | ((~R0v[3] >> 31) << 2) | may;
                }
                __syncthreads();
                const uint32_t eNext = has_next ? xE[xb][lg + 1][lr] : 0u;
                const uint32_t sNext = has_next && lr + 1u < kRegRows ? xS[xb][lg + 1][lr + 1] : 0u;
                // carry in from the previous group's last site, which flips with
                // this group's first E bit of this row and S bit of the row above
                uint32_t cin = 0u;
                if constexpr (kOneBarrier) {
                    if (lg > 0u) {
                        const uint32_t P = xC[xb][lg - 1][lr];
                        const uint32_t hz = S1[0] & P, vt = (P >> 1) & E[0], d = P >> 2;
                        cin = ((hz & d) | (vt & ~d)) & (P >> 3) & 1u;
                    }
                }
                uint32_t horiz[4], vert[4], live[4], any = 0u;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const uint32_t eHi = (w < 3) ? E[w + 1] : eNext;
                    const uint32_t sHi = (w < 3) ? S1[w + 1] : sNext;
                    const uint32_t sN = (S1[w] >> 1) | (sHi << 31);
                    const uint32_t sW = (E[w] >> 1) | (eHi << 31);
                    horiz[w] = sN & N[w];
                    vert[w] = W1[w] & sW;
                    live[w] = horiz[w] | vert[w];
                    any |= live[w];
                }
                uint32_t F[4] = {0u, 0u, 0u, 0u};
                if (act && lr + 1u < LR && any) {
                    uint32_t D[4];
                    decide_group<MODE>(key0, key1, (uint32_t)gg, (uint32_t)gr, t, c, Tall, R0v, vert, live, D);
#pragma unroll
                    for (int w = 0; w < 4; ++w) F[w] = (horiz[w] & D[w]) | (vert[w] & ~D[w]);
                }
                // own N and E planes (E shifted by one site)
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    N[w] ^= F[w];
                    E[w] ^= (F[w] << 1) | (w > 0 ? F[w - 1] >> 31 : 0u);
                }
                // the flips of the row above: this row's W and S planes (S shifted)
                uint32_t Fd[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) Fd[w] = lane_prev(F[w]);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    W[w] ^= Fd[w];
                    S[w] ^= (Fd[w] << 1) | (w > 0 ? Fd[w - 1] >> 31 : 0u);
                }
                if constexpr (kOneBarrier) {
                    E[0] ^= cin;
                    S[0] ^= lane_prev(cin);   // the carry of the row below
                } else {
                    xC[0][lg][lr] = F[3] >> 31;
                    __syncthreads();
                    if (lg > 0u) {
                        E[0] ^= xC[0][lg - 1][lr];
                        if (lr > 0u) S[0] ^= xC[0][lg - 1][lr - 1];
                    }
                }
                xb ^= 1u;
            }
        }
    }
    if (mine && lr >= HR && lr < HR + TR && lg >= HG && lg < HG + TG) {
        uint32_t *p = out + (size_t)gr * RS + 4 * gg;
        st4(p, N);
        st4(p + PS, S);
        st4(p + 2 * PS, E);
        st4(p + 3 * PS, W);
    }
}

// Multi-job kernel: work-group b runs tile items[b].tile of job items[b].job,
// with that job's plan, thresholds and key.
template <int MODE, bool RANDOM>
__device__ __forceinline__ void domino_item(uint32_t *lds, const TileJob &j, uint32_t tile)
{
    domino_tile<MODE, RANDOM>(lds, j.in, j.out, j.PS, j.RS, j.ng, j.rows, (uint32_t)j.omega, j.t0, j.S, j.TR, j.TG,
                              j.HR, j.HG, tile / j.tiles_x, tile % j.tiles_x, j.T, j.key0, j.key1);
}

// Every job of a launch has the colour order RANDOM.
template <bool RANDOM>
__global__ void __launch_bounds__(1024) domino_items_kernel(const TileJob *__restrict__ jobs,
                                                            const TileItem *__restrict__ items)
{
    extern __shared__ uint32_t lds[];
    const TileItem it = items[blockIdx.x];
    const TileJob &j = jobs[it.job];
    if (j.mode == kUniform)
        domino_item<kUniform, RANDOM>(lds, j, it.tile);
    else if (j.mode == kMetropolis)
        domino_item<kMetropolis, RANDOM>(lds, j, it.tile);
    else
        domino_item<kHeatBath, RANDOM>(lds, j, it.tile);
}

// ------------------------------------------------------------ batched chains
// Persistent kernel over a list of bundles of independent chains (costliest
// first).  A work-group takes the next bundle from an atomic counter, copies
// the whole state of each member into LDS (compact rows of 4*ng words, n rows,
// no padding, members back to back), runs all nsweeps sweeps there and writes
// the members back.  Several small chains share a work-group, so a chain too
// small to keep a CU busy no longer holds one alone.  Every work-group leaves
// the loop once the counter passes the end of the list.
__global__ void batch_reset_kernel(uint32_t *counter) { *counter = 0u; }

template <int MODE, bool RANDOM>
__global__ void __launch_bounds__(1024) domino_batch_kernel(BatchChain *chains, const BatchBundle *bundles,
                                                            const uint32_t *members, uint32_t nbundles,
                                                            uint32_t *counter, uint32_t *planes, uint32_t nsweeps,
                                                            Thr Tall)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_next;
    __shared__ uint32_t s_first[kBundleMax + 1];   // first task of each member (prefix of n * ng)
    __shared__ uint32_t s_off[kBundleMax];         // LDS word offset of each member
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    for (;;) {
        if (tid == 0) s_next = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t bi = s_next;
        __syncthreads();
        if (bi >= nbundles) return;
        const BatchBundle B = bundles[bi];
        if (tid == 0) {
            uint32_t task = 0, off = 0;
            for (uint32_t k = 0; k < B.count; ++k) {
                const BatchChain &ch = chains[members[B.first + k]];
                s_first[k] = task;
                s_off[k] = off;
                task += ch.n * ch.ng;
                off += 4u * ch.n * 4u * ch.ng;
            }
            s_first[B.count] = task;
        }
        __syncthreads();
        // load every member (compact rows: 4 ng words, n rows, 4 planes)
        for (uint32_t k = 0; k < B.count; ++k) {
            const BatchChain ch = chains[members[B.first + k]];
            const uint32_t LRS = 4 * ch.ng, LPS = ch.n * LRS, items = 4 * ch.n * ch.ng;
            const uint32_t *g = planes + ch.offset;
            uint32_t *l = lds + s_off[k];
            for (uint32_t j = tid; j < items; j += nt) {
                const uint32_t gg = j % ch.ng, r = (j / ch.ng) % ch.n, p = j / (ch.ng * ch.n);
                uint32_t v[4];
                ld4(g + p * ch.PS + (size_t)r * ch.RS + 4 * gg, v);
                st4(l + p * LPS + r * LRS + 4 * gg, v);
            }
        }
        __syncthreads();
        if (B.count == 1) {
            // one chain, as many passes over its (row, group) tasks as needed
            const BatchChain ch = chains[members[B.first]];
            const uint32_t n = ch.n, ng = ch.ng, LRS = 4 * ng, LPS = n * LRS, omega = (n + 1) & 1u;
            const uint32_t tasks = n * ng;
            for (uint32_t s = 0; s < nsweeps; ++s) {
                for (uint32_t i = 0; i < 2; ++i) {
                    uint32_t c = i, t = ch.t + s;
                    if constexpr (RANDOM) {
                        t = 2u * t + i;
                        c = step_colour(t, 2u, ch.key0, ch.key1);
                    }
                    for (uint32_t task = tid; task < tasks; task += nt) {
                        const uint32_t r = task / ng, gg = task % ng;
                        uint32_t *pN = lds + r * LRS + 4 * gg;
                        if (c == omega)
                            owner_group<MODE>(pN, pN + LPS, pN + 2 * LPS, pN + 3 * LPS, r, gg, c, t, Tall, ch.key0,
                                              ch.key1);
                        else if (r + 1 < n)
                            other_group<MODE>(pN, pN + 2 * LPS, pN + LPS + LRS, pN + 3 * LPS + LRS, r, gg, c, t, Tall,
                                              ch.key0, ch.key1, gg + 1 < ng);
                    }
                    __syncthreads();
                }
            }
        } else {
            // several small chains side by side: one task per thread
            const bool has = tid < s_first[B.count];
            uint32_t k = 0;
            while (has && k + 1 < B.count && tid >= s_first[k + 1]) ++k;
            const BatchChain ch = chains[members[B.first + k]];
            const uint32_t n = ch.n, ng = ch.ng, LRS = 4 * ng, LPS = n * LRS, omega = (n + 1) & 1u;
            const uint32_t local = tid - s_first[k], r = local / ng, gg = local % ng;
            uint32_t *pN = lds + s_off[k] + r * LRS + 4 * gg;
            for (uint32_t s = 0; s < nsweeps; ++s) {
                for (uint32_t i = 0; i < 2; ++i) {
                    uint32_t c = i, t = ch.t + s;
                    if constexpr (RANDOM) {
                        t = 2u * t + i;
                        c = step_colour(t, 2u, ch.key0, ch.key1);
                    }
                    if (has) {
                        if (c == omega)
                            owner_group<MODE>(pN, pN + LPS, pN + 2 * LPS, pN + 3 * LPS, r, gg, c, t, Tall, ch.key0,
                                              ch.key1);
                        else if (r + 1 < n)
                            other_group<MODE>(pN, pN + 2 * LPS, pN + LPS + LRS, pN + 3 * LPS + LRS, r, gg, c, t, Tall,
                                              ch.key0, ch.key1, gg + 1 < ng);
                    }
                    __syncthreads();
                }
            }
        }
        for (uint32_t k = 0; k < B.count; ++k) {
            const uint32_t ci = members[B.first + k];
            const BatchChain ch = chains[ci];
            const uint32_t LRS = 4 * ch.ng, LPS = ch.n * LRS, items = 4 * ch.n * ch.ng;
            uint32_t *g = planes + ch.offset;
            const uint32_t *l = lds + s_off[k];
            for (uint32_t j = tid; j < items; j += nt) {
                const uint32_t gg = j % ch.ng, r = (j / ch.ng) % ch.n, p = j / (ch.ng * ch.n);
                uint32_t v[4];
                ld4(l + p * LPS + r * LRS + 4 * gg, v);
                st4(g + p * ch.PS + (size_t)r * ch.RS + 4 * gg, v);
            }
            if (tid == 0) chains[ci].t = ch.t + nsweeps;
        }
        __syncthreads();
    }
}

// Crossing bit of an owner's edge plane p at box vertex (P, Q) (0 outside).
__device__ __forceinline__ uint32_t owner_bit(const uint32_t *planes, size_t PS, uint32_t RS, int n, int p, int P,
                                              int Q)
{
    const int r2 = P + Q - n - 1, k2 = Q - P + n - 1;
    if (r2 < 0 || k2 < 0) return 0u;
    const int r = r2 >> 1, k = k2 >> 1;
    if (r >= n || k >= n) return 0u;
    return (planes[(size_t)p * PS + (size_t)r * RS + (k >> 5)] >> (k & 31)) & 1u;
}

// Horizontal segment (P,Q)-(P+1,Q) and vertical segment (P,Q)-(P,Q+1).
__device__ __forceinline__ uint32_t hseg(const uint32_t *pl, size_t PS, uint32_t RS, int n, int om, int P, int Q)
{
    return (((P + Q) & 1) == om) ? owner_bit(pl, PS, RS, n, 2, P, Q) : owner_bit(pl, PS, RS, n, 3, P + 1, Q);
}
__device__ __forceinline__ uint32_t vseg(const uint32_t *pl, size_t PS, uint32_t RS, int n, int om, int P, int Q)
{
    return (((P + Q) & 1) == om) ? owner_bit(pl, PS, RS, n, 0, P, Q) : owner_bit(pl, PS, RS, n, 1, P, Q + 1);
}

__device__ __forceinline__ bool face_in(int n, int X, int Y)
{
    return abs(2 * X - 2 * n + 1) + abs(2 * Y - 2 * n + 1) <= 2 * n;
}

// Faces (x, y) of a w x h box at face offset (ox, oy) in the diamond's box
// (the whole 2n x 2n box for the Aztec diamond).  Uncovered faces (outside the
// diamond, or outside a domain inside it) have no crossed edge: 0xFF.
__global__ void domino_export_kernel(const uint32_t *pl, size_t PS, uint32_t RS, int n, int om, int ox, int oy,
                                     int w, int h, uint8_t *faces)
{
    const int x = blockIdx.x * 16 + threadIdx.x, y = blockIdx.y * 16 + threadIdx.y;
    if (x >= w || y >= h) return;
    const int X = x + ox, Y = y + oy;
    uint8_t d = 0xFF;
    if (face_in(n, X, Y)) {
        if (hseg(pl, PS, RS, n, om, X, Y + 1)) d = 0;
        else if (hseg(pl, PS, RS, n, om, X, Y)) d = 1;
        else if (vseg(pl, PS, RS, n, om, X + 1, Y)) d = 2;
        else if (vseg(pl, PS, RS, n, om, X, Y)) d = 3;
    }
    faces[(size_t)y * w + x] = d;
}

// Faces covered by horizontal dominoes = the two faces beside every crossed
// vertical edge, i.e. beside the crossed N and S edges of the owners.  One
// thread per owner word; owner (r, k) is box vertex (X, Y) = (r-k+n, r+k+1):
// a crossed N edge covers faces (X-1, Y) and (X, Y), a crossed S edge faces
// (X-1, Y-1) and (X, Y-1).  Counts go to a block-local copy of the bins in LDS
// (when they fit) and are flushed with one global atomic per touched bin.
// Bins cover the box of a domain at face offset (ox, oy) (0 for the Aztec
// diamond); the run-counting path below assumes offset 0.
constexpr uint32_t kLdsBins = 8192;

__global__ void __launch_bounds__(1024) domino_observe_kernel(const uint32_t *pl, size_t PS, uint32_t RS, int n,
                                                             uint32_t nw, uint32_t B, uint32_t bins_x,
                                                             uint32_t nbins, int ox, int oy,
                                                             unsigned long long *bins)
{
    extern __shared__ uint32_t lbin[];
    const bool local = nbins <= kLdsBins;
    if (local) {
        for (uint32_t i = threadIdx.x; i < nbins; i += blockDim.x) lbin[i] = 0u;
        __syncthreads();
    }
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = gid / nw, w = gid % nw;
    if (r < (uint32_t)n) {
        for (int p = 0; p < 2; ++p) {
            uint32_t m = pl[(size_t)p * PS + (size_t)r * RS + w];
            if (B >= 32u && ox == 0 && oy == 0) {
                // site k = 32w + b sits at X = X0 - b, Y = Y0 + b: with bins of
                // at least 32 faces, the word's bits fall into at most three
                // runs per face column (X - 1 and X), each one bin
                if (!m) continue;
                const int X0 = (int)r - (int)(w * 32u) + n, Y0 = (int)r + (int)(w * 32u) + 1 - p;
                const uint32_t yb0 = (uint32_t)Y0 / B, ybrk = B - (uint32_t)Y0 % B;
                for (int d = 1; d >= 0; --d) {
                    const uint32_t c0 = (uint32_t)(X0 - d), xb0 = c0 / B, xbrk = c0 % B + 1u;
                    const uint32_t s1 = ybrk < xbrk ? ybrk : xbrk, s2 = ybrk < xbrk ? xbrk : ybrk;
                    const uint32_t cuts[4] = {0u, s1 < 32u ? s1 : 32u, s2 < 32u ? s2 : 32u, 32u};
                    for (int q = 0; q < 3; ++q) {
                        const uint32_t lo = cuts[q], hi = cuts[q + 1];
                        if (lo >= hi) continue;
                        const uint32_t mask = (hi >= 32u ? ~0u : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
                        const uint32_t cnt = (uint32_t)__popc(m & mask);
                        if (!cnt) continue;
                        const uint32_t i = (yb0 + (lo >= ybrk ? 1u : 0u)) * bins_x + xb0 - (lo >= xbrk ? 1u : 0u);
                        if (local)
                            atomicAdd(&lbin[i], cnt);
                        else
                            atomicAdd(&bins[i], (unsigned long long)cnt);
                    }
                }
                continue;
            }
            while (m) {
                const int b = __builtin_ctz(m);
                m &= m - 1u;
                const int k = (int)(w * 32u) + b;
                const int X = (int)r - k + n - ox, Y = (int)r + k + 1 - p - oy;   // face row of the crossed edge
                const uint32_t i0 = (uint32_t)(Y / (int)B) * bins_x + (uint32_t)((X - 1) / (int)B);
                const uint32_t i1 = (uint32_t)(Y / (int)B) * bins_x + (uint32_t)(X / (int)B);
                if (local) {
                    atomicAdd(&lbin[i0], 1u);
                    atomicAdd(&lbin[i1], 1u);
                } else {
                    atomicAdd(&bins[i0], 1ull);
                    atomicAdd(&bins[i1], 1ull);
                }
            }
        }
    }
    if (local) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nbins; i += blockDim.x)
            if (lbin[i]) atomicAdd(&bins[i], (unsigned long long)lbin[i]);
    }
}

}  // namespace

hipError_t domino_init(const DominoDev &d, int init_max, hipStream_t s)
{
    dim3 block(64), grid((d.RS + 63) / 64, d.n + 1);
    hipLaunchKernelGGL(domino_init_kernel, grid, block, 0, s, d.planes, d.spare, d.PS, d.RS, d.n, init_max);
    return hipGetLastError();
}

hipError_t domino_colour_step(const DominoDev &d, int colour, uint32_t t, const Thr &T, int metropolis,
                              uint64_t seed, hipStream_t s, Timing *tm)
{
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t threads = d.ng * (uint32_t)d.n;
    dim3 block(256), grid((threads + 255) / 256);
    const bool owner = colour == d.omega;
    const uint32_t n = (uint32_t)d.n, c = (uint32_t)colour;
    if (owner)
    {
        auto k = T.uniform() ? domino_owner_step<kUniform>
                             : (metropolis ? domino_owner_step<kMetropolis> : domino_owner_step<kHeatBath>);
        return launch(tm, 1, k, grid, block, 0, s, d.planes, d.PS, d.RS, d.ng, n, c, t, T, key0, key1);
    }
    auto k = T.uniform() ? domino_other_step<kUniform>
                         : (metropolis ? domino_other_step<kMetropolis> : domino_other_step<kHeatBath>);
    return launch(tm, 1, k, grid, block, 0, s, d.planes, d.PS, d.RS, d.ng, n, c, t, T, key0, key1);
}

DominoTile domino_auto_tile(int n, bool random_order, bool weighted)
{
    DominoTile t;
    uint32_t ng, RS;
    size_t PS;
    domino_words(n, &ng, &RS, &PS);
    if ((uint32_t)n <= 128 && ng <= 4) {   // whole domain in one tile, no halo
        t.TR = (uint32_t)n;
        t.TG = ng;
        t.S = 1u << 30;
        return t;
    }
    // register tiles of 64 lanes: 32 owned rows and a halo of 16 sweeps (8
    // under the random colour order, two halo rows per sweep); measured on
    // MI355X for order 2048: 2 groups wide for one-bit decisions, 4 for
    // bit-serial ones
    t.reg = 1;
    t.TR = 32;
    t.TG = weighted && !random_order ? (ng < 4 ? ng : 4) : (ng < 2 ? ng : 2);
    t.S = random_order ? 8 : 16;
    return t;
}

bool domino_plan(const DominoDev &d, const DominoTile &tile, uint32_t S_max, TilePlan *p)
{
    const uint32_t n = (uint32_t)d.n;
    if (n == 0 || S_max == 0) return false;
    const uint32_t TG = tile.TG == 0 ? 1u : (tile.TG < d.ng ? tile.TG : d.ng);
    const uint32_t tiles_x = (d.ng + TG - 1) / TG;
    const uint32_t LG0 = TG + (tiles_x > 1 ? 2u : 0u);
    // one thread per (row, group) task; register tiles: a wavefront of 64
    // rows per group
    const uint32_t max_rows = tile.reg ? kRegRows : 1024u / LG0;
    if (tile.reg && LG0 > kRegGroups) return false;
    // halo rows per sweep: 1 (one step of the other colour), 2 under the
    // random colour order (any step may be of the other colour)
    const uint32_t hps = tile.order ? 2u : 1u;
    if (max_rows < 2u * hps + 1u) return false;
    uint32_t TR = tile.TR == 0 ? 1u : (tile.TR < n ? tile.TR : n);
    // leave room for a halo of one sweep on each side
    if (TR < n && TR > max_rows - 2u * hps) TR = max_rows - 2u * hps;
    if (TR >= n && n > max_rows) TR = max_rows - 2u * hps;
    const uint32_t tiles_y = (n + TR - 1) / TR;
    uint32_t S = S_max < tile.S ? S_max : tile.S;
    if (tiles_x > 1 && S * hps > 128u) S = 128u / hps;   // the one-group column halo covers 128 steps
    if (tiles_y > 1 && S * hps > (max_rows - TR) / 2u) S = (max_rows - TR) / 2u / hps;
    if (S == 0u) S = 1u;
    const uint32_t HR = tiles_y > 1 ? hps * S : 0u;
    const uint32_t HG = tiles_x > 1 ? 1u : 0u;
    const uint32_t LR = TR + 2 * HR, LG = TG + 2 * HG;
    const uint32_t tasks = LR * LG;
    const uint32_t lds = 4u * LR * domino_lds_row_words(LG) * 4u;
    if (tasks > 1024u || lds > 160u * 1024u) return false;
    p->S = S;
    p->TR = TR;
    p->TG = TG;
    p->HR = HR;
    p->HG = HG;
    p->tiles_x = tiles_x;
    p->tiles_y = tiles_y;
    p->threads = tile.reg ? LG * kRegRows : (tasks + 63) / 64 * 64;
    p->lds = tile.reg ? 0u : lds;
    p->order = tile.order;
    p->reg = tile.reg;
    return true;
}

hipError_t domino_tiled_sweeps(DominoDev &d, const DominoTile &tile, uint32_t t0, uint32_t nsw, const Thr &T,
                               int metropolis, uint64_t seed, hipStream_t s, Timing *tm)
{
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    uint32_t done = 0;
    while (done < nsw) {
        TilePlan p;
        if (!domino_plan(d, tile, nsw - done, &p)) return hipErrorInvalidConfiguration;
#define TL_DOMINO_PICK(KERNEL)                                                                        \
    (p.order ? (T.uniform() ? KERNEL<kUniform, true>                                                  \
                            : (metropolis ? KERNEL<kMetropolis, true> : KERNEL<kHeatBath, true>))    \
             : (T.uniform() ? KERNEL<kUniform, false>                                                 \
                            : (metropolis ? KERNEL<kMetropolis, false> : KERNEL<kHeatBath, false>)))
        auto k = p.reg ? TL_DOMINO_PICK(domino_reg_kernel) : TL_DOMINO_PICK(domino_tiled_kernel);
#undef TL_DOMINO_PICK
        hipError_t e = launch(tm, 2 * p.S, k, dim3(p.tiles()), dim3(p.threads), p.lds, s, (const uint32_t *)d.planes,
                              d.spare, d.PS, d.RS, d.ng, (uint32_t)d.n, (uint32_t)d.omega, t0 + done, p.S, p.TR,
                              p.TG, p.HR, p.HG, p.tiles_x, T, key0, key1);
        if (e != hipSuccess) return e;
        uint32_t *tmp = d.planes;
        d.planes = d.spare;
        d.spare = tmp;
        done += p.S;
    }
    return hipSuccess;
}

TileJob domino_tile_job(const DominoDev &d, const TilePlan &p, uint32_t t0, const Thr &T, int metropolis,
                        uint64_t seed)
{
    TileJob j{};
    j.in = d.planes;
    j.out = d.spare;
    j.PS = d.PS;
    j.RS = d.RS;
    j.ng = d.ng;
    j.rows = (uint32_t)d.n;
    j.P = 4;
    j.omega = d.omega;
    j.t0 = t0;
    j.S = p.S;
    j.TR = p.TR;
    j.TG = p.TG;
    j.HR = p.HR;
    j.HG = p.HG;
    j.tiles_x = p.tiles_x;
    j.order = p.order;
    j.mode = T.uniform() ? kModeUniform : (metropolis ? kModeMetropolis : kModeHeatBath);
    j.key0 = (uint32_t)seed;
    j.key1 = (uint32_t)(seed >> 32);
    j.T = T;
    return j;
}

hipError_t domino_items(const TileJob *jobs, const TileItem *items, uint32_t n_items, uint32_t threads, uint32_t lds,
                        uint32_t order, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (threads == 0 || threads > 1024u || lds > 160u * 1024u) return hipErrorInvalidConfiguration;
    if (order)
        hipLaunchKernelGGL(domino_items_kernel<true>, dim3(n_items), dim3(threads), lds, s, jobs, items);
    else
        hipLaunchKernelGGL(domino_items_kernel<false>, dim3(n_items), dim3(threads), lds, s, jobs, items);
    return hipGetLastError();
}

hipError_t domino_batch_sweeps(BatchChain *chains, const BatchBundle *bundles, const uint32_t *members,
                               uint32_t nbundles, uint32_t *counter, uint32_t *planes, uint32_t nsweeps, const Thr &T,
                               int metropolis, uint32_t colour_order, uint32_t threads, uint32_t workgroups,
                               uint32_t lds_bytes, hipStream_t s, Timing *tm)
{
    if (threads == 0 || threads > 1024 || (threads & 63) || lds_bytes > 160u * 1024u - 64u)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    auto k = colour_order
                 ? (T.uniform() ? domino_batch_kernel<kUniform, true>
                                : (metropolis ? domino_batch_kernel<kMetropolis, true>
                                              : domino_batch_kernel<kHeatBath, true>))
                 : (T.uniform() ? domino_batch_kernel<kUniform, false>
                                : (metropolis ? domino_batch_kernel<kMetropolis, false>
                                              : domino_batch_kernel<kHeatBath, false>));
    return launch(tm, 2 * nsweeps, k, dim3(workgroups), dim3(threads), lds_bytes, s, chains, bundles, members,
                  nbundles, counter, planes, nsweeps, T);
}

hipError_t domino_export(const DominoDev &d, uint8_t *faces, hipStream_t s)
{
    return domino_export_box(d, 0, 0, 2 * d.n, 2 * d.n, faces, s);
}

hipError_t domino_export_box(const DominoDev &d, int ox, int oy, int w, int h, uint8_t *faces, hipStream_t s)
{
    dim3 block(16, 16), grid((w + 15) / 16, (h + 15) / 16);
    hipLaunchKernelGGL(domino_export_kernel, grid, block, 0, s, d.planes, d.PS, d.RS, d.n, d.omega, ox, oy, w, h,
                       faces);
    return hipGetLastError();
}

hipError_t domino_observe(const DominoDev &d, uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s)
{
    return domino_observe_box(d, 0, 0, 2 * d.n, B, bins_x, bins, s);
}

hipError_t domino_observe_box(const DominoDev &d, int ox, int oy, int h, uint32_t B, uint32_t bins_x,
                              unsigned long long *bins, hipStream_t s)
{
    const uint32_t nw = (uint32_t)((d.n + 31) / 32);
    const uint32_t bins_y = ((uint32_t)h + B - 1) / B;
    const uint32_t nbins = bins_x * bins_y;
    const uint32_t threads = nw * (uint32_t)d.n;
    // counting runs of a word (bins of 32 faces or more, no offset): large
    // work-groups, each clearing and flushing the LDS bins once; single
    // dominoes: smaller ones, so that fewer lanes share a block's bins
    const uint32_t bs = B >= 32u && ox == 0 && oy == 0 ? 1024u : 256u;
    dim3 block(bs), grid((threads + bs - 1) / bs);
    const uint32_t shmem = nbins <= kLdsBins ? nbins * 4u : 0u;
    hipLaunchKernelGGL(domino_observe_kernel, grid, block, shmem, s, d.planes, d.PS, d.RS, d.n, nw, B, bins_x, nbins,
                       ox, oy, bins);
    return hipGetLastError();
}

}  // namespace tl
