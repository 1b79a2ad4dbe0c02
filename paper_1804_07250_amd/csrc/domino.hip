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

__global__ void domino_init_kernel(uint32_t *planes, size_t PS, uint32_t RS, int n, int init_max)
{
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = blockIdx.y;
    if (w >= RS || r > (uint32_t)n) return;
    uint32_t bits[4] = {0u, 0u, 0u, 0u};
    if (r < (uint32_t)n) {
        for (int b = 0; b < 32; ++b) {
            const int k = (int)(w * 32u) + b;
            if (k >= n) break;
            const int x = (int)r - k, y = (int)r + k + 1 - n;
            if (!init_max) {        // horizontal brick: N and S edges
                bits[0] |= brick_pair(n, x, y) << b;
                bits[1] |= brick_pair(n, x, y - 1) << b;
            } else {                // vertical brick (the transpose): E and W edges
                bits[2] |= brick_pair(n, y, x) << b;
                bits[3] |= brick_pair(n, y, x - 1) << b;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) planes[p * PS + (size_t)r * RS + w] = bits[p];
}

__device__ __forceinline__ uint4 ld4(const uint32_t *p) { return *reinterpret_cast<const uint4 *>(p); }
__device__ __forceinline__ void st4(uint32_t *p, const uint32_t (&v)[4])
{
    *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void unpack(uint4 q, uint32_t (&v)[4])
{
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
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

// One colour step of the owner colour: all bits local to the owner.
template <bool METRO>
__global__ void __launch_bounds__(256) domino_owner_step(uint32_t *planes, size_t PS, uint32_t RS,
                                                         uint32_t ng, uint32_t n, uint32_t c,
                                                         uint32_t t, Thr Tall, uint32_t key0,
                                                         uint32_t key1)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t g = gid % ng, r = gid / ng;
    if (r >= n) return;
    uint32_t *base = planes + (size_t)r * RS + 4u * g;
    uint32_t N[4], S[4], E[4], W[4];
    unpack(ld4(base), N);
    unpack(ld4(base + PS), S);
    unpack(ld4(base + 2 * PS), E);
    unpack(ld4(base + 3 * PS), W);
    uint32_t horiz[4], vert[4], live[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        horiz[w] = N[w] & S[w];
        vert[w] = E[w] & W[w];
        live[w] = horiz[w] | vert[w];
    }
    if ((live[0] | live[1] | live[2] | live[3]) == 0u) return;
    constexpr int NC = DomCtx<METRO>::NC;
    uint32_t T[NC], cm[NC][4], D[4];
    DomCtx<METRO>::build(r, c, Tall, vert, T, cm);
    decide128<NC>(key0, key1, g, r, t, c, T, cm, live, D);
    uint32_t F[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        F[w] = (horiz[w] & D[w]) | (vert[w] & ~D[w]);
        N[w] ^= F[w];
        S[w] ^= F[w];
        E[w] ^= F[w];
        W[w] ^= F[w];
    }
    st4(base, N);
    st4(base + PS, S);
    st4(base + 2 * PS, E);
    st4(base + 3 * PS, W);
}

// One colour step of the other colour.  Its site (r, k) uses bits N(r,k),
// W(r+1,k) (aligned) and S(r+1,k+1), E(r,k+1) (shifted by one bit).  Bit 0 of
// the first word of a group in the shifted planes belongs to the previous
// group's last site, so the first and carry words are updated atomically.
template <bool METRO>
__global__ void __launch_bounds__(256) domino_other_step(uint32_t *planes, size_t PS, uint32_t RS,
                                                         uint32_t ng, uint32_t n, uint32_t c,
                                                         uint32_t t, Thr Tall, uint32_t key0,
                                                         uint32_t key1)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t g = gid % ng, r = gid / ng;
    if (r + 1u >= n) return;   // the other colour has rows 0 .. n-2
    uint32_t *rowN = planes + (size_t)r * RS + 4u * g;
    uint32_t *rowE = planes + 2 * PS + (size_t)r * RS + 4u * g;
    uint32_t *rowS1 = planes + PS + (size_t)(r + 1) * RS + 4u * g;
    uint32_t *rowW1 = planes + 3 * PS + (size_t)(r + 1) * RS + 4u * g;
    uint32_t oN[4], oE[4], oS1[4], oW1[4];
    unpack(ld4(rowN), oN);
    unpack(ld4(rowE), oE);
    unpack(ld4(rowS1), oS1);
    unpack(ld4(rowW1), oW1);
    const uint32_t eNext = rowE[4], sNext = rowS1[4];
    uint32_t sN[4], sS[4], sE[4], sW[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t eHi = (w < 3) ? oE[w + 1] : eNext;
        const uint32_t sHi = (w < 3) ? oS1[w + 1] : sNext;
        sS[w] = oN[w];
        sE[w] = oW1[w];
        sN[w] = (oS1[w] >> 1) | (sHi << 31);
        sW[w] = (oE[w] >> 1) | (eHi << 31);
    }
    uint32_t horiz[4], vert[4], live[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        horiz[w] = sN[w] & sS[w];
        vert[w] = sE[w] & sW[w];
        live[w] = horiz[w] | vert[w];
    }
    if ((live[0] | live[1] | live[2] | live[3]) == 0u) return;
    constexpr int NC = DomCtx<METRO>::NC;
    uint32_t T[NC], cm[NC][4], D[4];
    DomCtx<METRO>::build(r, c, Tall, vert, T, cm);
    decide128<NC>(key0, key1, g, r, t, c, T, cm, live, D);
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
    if (F[3] >> 31) {
        atomicXor(&rowE[4], 1u);
        atomicXor(&rowS1[4], 1u);
    }
}

// Crossing bit of an owner's edge plane p at box vertex (P, Q) (0 outside).
__device__ __forceinline__ uint32_t owner_bit(const uint32_t *planes, size_t PS, uint32_t RS, int n,
                                              int p, int P, int Q)
{
    const int r2 = P + Q - n - 1, k2 = Q - P + n - 1;
    if (r2 < 0 || k2 < 0) return 0u;
    const int r = r2 >> 1, k = k2 >> 1;
    if (r >= n || k >= n) return 0u;
    return (planes[(size_t)p * PS + (size_t)r * RS + (k >> 5)] >> (k & 31)) & 1u;
}

// Horizontal segment (P,Q)-(P+1,Q) and vertical segment (P,Q)-(P,Q+1).
__device__ __forceinline__ uint32_t hseg(const uint32_t *pl, size_t PS, uint32_t RS, int n, int om, int P,
                                         int Q)
{
    return (((P + Q) & 1) == om) ? owner_bit(pl, PS, RS, n, 2, P, Q) : owner_bit(pl, PS, RS, n, 3, P + 1, Q);
}
__device__ __forceinline__ uint32_t vseg(const uint32_t *pl, size_t PS, uint32_t RS, int n, int om, int P,
                                         int Q)
{
    return (((P + Q) & 1) == om) ? owner_bit(pl, PS, RS, n, 0, P, Q) : owner_bit(pl, PS, RS, n, 1, P, Q + 1);
}

__device__ __forceinline__ bool face_in(int n, int X, int Y)
{
    return abs(2 * X - 2 * n + 1) + abs(2 * Y - 2 * n + 1) <= 2 * n;
}

__global__ void domino_export_kernel(const uint32_t *pl, size_t PS, uint32_t RS, int n, int om,
                                     uint8_t *faces)
{
    const int X = blockIdx.x * 16 + threadIdx.x, Y = blockIdx.y * 16 + threadIdx.y;
    if (X >= 2 * n || Y >= 2 * n) return;
    uint8_t d = 0xFF;
    if (face_in(n, X, Y)) {
        if (hseg(pl, PS, RS, n, om, X, Y + 1)) d = 0;
        else if (hseg(pl, PS, RS, n, om, X, Y)) d = 1;
        else if (vseg(pl, PS, RS, n, om, X + 1, Y)) d = 2;
        else if (vseg(pl, PS, RS, n, om, X, Y)) d = 3;
    }
    faces[(size_t)Y * (2 * n) + X] = d;
}

// Per face: covered by a horizontal domino (one of its vertical sides crossed).
__global__ void domino_observe_kernel(const uint32_t *pl, size_t PS, uint32_t RS, int n, int om,
                                      uint32_t B, uint32_t bins_x, unsigned long long *bins)
{
    const int X = blockIdx.x * 16 + threadIdx.x, Y = blockIdx.y * 16 + threadIdx.y;
    const bool valid = X < 2 * n && Y < 2 * n && face_in(n, X, Y);
    uint64_t q = 0;
    if (valid) q = vseg(pl, PS, RS, n, om, X, Y) | vseg(pl, PS, RS, n, om, X + 1, Y);
    bin_add(q, X, Y, valid, B, bins_x, bins);
}

}  // namespace

hipError_t domino_init(const DominoDev &d, int init_max, hipStream_t s)
{
    dim3 block(64), grid((d.RS + 63) / 64, d.n + 1);
    hipLaunchKernelGGL(domino_init_kernel, grid, block, 0, s, d.planes, d.PS, d.RS, d.n, init_max);
    return hipGetLastError();
}

hipError_t domino_colour_step(const DominoDev &d, int colour, uint32_t t, const Thr &T, int metropolis,
                              uint64_t seed, hipStream_t s)
{
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t threads = d.ng * (uint32_t)d.n;
    dim3 block(256), grid((threads + 255) / 256);
    const bool owner = colour == d.omega;
    if (owner) {
        if (metropolis)
            hipLaunchKernelGGL(domino_owner_step<true>, grid, block, 0, s, d.planes, d.PS, d.RS, d.ng,
                               (uint32_t)d.n, (uint32_t)colour, t, T, key0, key1);
        else
            hipLaunchKernelGGL(domino_owner_step<false>, grid, block, 0, s, d.planes, d.PS, d.RS, d.ng,
                               (uint32_t)d.n, (uint32_t)colour, t, T, key0, key1);
    } else {
        if (metropolis)
            hipLaunchKernelGGL(domino_other_step<true>, grid, block, 0, s, d.planes, d.PS, d.RS, d.ng,
                               (uint32_t)d.n, (uint32_t)colour, t, T, key0, key1);
        else
            hipLaunchKernelGGL(domino_other_step<false>, grid, block, 0, s, d.planes, d.PS, d.RS, d.ng,
                               (uint32_t)d.n, (uint32_t)colour, t, T, key0, key1);
    }
    return hipGetLastError();
}

hipError_t domino_export(const DominoDev &d, uint8_t *faces, hipStream_t s)
{
    dim3 block(16, 16), grid((2 * d.n + 15) / 16, (2 * d.n + 15) / 16);
    hipLaunchKernelGGL(domino_export_kernel, grid, block, 0, s, d.planes, d.PS, d.RS, d.n, d.omega, faces);
    return hipGetLastError();
}

hipError_t domino_observe(const DominoDev &d, uint32_t B, uint32_t bins_x, unsigned long long *bins,
                          hipStream_t s)
{
    dim3 block(16, 16), grid((2 * d.n + 15) / 16, (2 * d.n + 15) / 16);
    hipLaunchKernelGGL(domino_observe_kernel, grid, block, 0, s, d.planes, d.PS, d.RS, d.n, d.omega, B,
                       bins_x, bins);
    return hipGetLastError();
}

}  // namespace tl
