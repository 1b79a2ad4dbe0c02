// Device-side building blocks shared by the three models: the Philox4x32-10
// generator, the bit-serial acceptance test "u < T" over 128 sites, and the
// observable bin reduction.  gfx950 only; wavefront size 64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tl {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products; the key (uniform across the wavefront, so it lives in
// scalar registers) is bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        // one 32 x 32 -> 64-bit product each (a single v_mad_u64_u32, where
        // separate high and low halves cost two multiplies), and each
        // three-way XOR as one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0, p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Colour of colour step `step` under the random colour order: floor(K u / 2^32)
// with u word 0 of Philox(ctr = (step, 0, 0, 2^31)); no site draw uses that
// counter (their last word is below 128).
__device__ __forceinline__ uint32_t step_colour(uint32_t step, uint32_t K, uint32_t k0, uint32_t k1)
{
    uint32_t out[4];
    philox4x32_10(step, 0u, 0u, 0x80000000u, k0, k1, out);
    return (uint32_t)(((uint64_t)out[0] * K) >> 32);
}

// Acceptance decisions for the 128 sites k = 128 g + 32 w + b (w = 0..3,
// b = 0..31) of class row r in colour step (t, c): bit b of D[w] is 1 iff the
// site's uniform u is below the threshold of its context.
//
// u is defined plane by plane from its most significant bit: bit 31-j of u is
// bit b of word w of Philox(ctr = (g, r, t, 4j + c)).  The comparison runs
// bit-serially from plane 0; a site leaves the loop as soon as its prefix of u
// differs from the prefix of its threshold, or when the threshold has no 1 bit
// left below the current plane.  Only the sites in `live` need a decision
// (the others are not flippable), so with T = 2^31 a single Philox call decides
// 128 sites.
//
// Contexts: site (w, b) is in context i iff bit b of cm[i][w] is set; the masks
// of one word partition (at least) the live sites.
template <int NC, uint32_t kDecidePlanes = 1>
__device__ __forceinline__ void decide128(uint32_t key0, uint32_t key1, uint32_t g, uint32_t r,
                                          uint32_t t, uint32_t c, const uint32_t (&T)[NC],
                                          const uint32_t (&cm)[NC][4], const uint32_t (&live)[4],
                                          uint32_t (&D)[4])
{
    uint32_t eq[4], lt[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        eq[w] = live[w];
        lt[w] = 0u;
    }
    // kDecidePlanes planes per iteration (a divisor of 32): their generator
    // calls are independent, so they overlap; a plane past the last undecided
    // site changes nothing.  Two pay off where the generator dominates (one
    // context), one elsewhere.
    static_assert(32u % kDecidePlanes == 0u, "planes per iteration divide 32");
    for (uint32_t j0 = 0; j0 < 32u; j0 += kDecidePlanes) {
        if ((eq[0] | eq[1] | eq[2] | eq[3]) == 0u) break;
        uint32_t R[kDecidePlanes][4];
#pragma unroll
        for (uint32_t u = 0; u < kDecidePlanes; ++u) philox4x32_10(g, r, t, ((j0 + u) << 2) | c, key0, key1, R[u]);
#pragma unroll
        for (uint32_t u = 0; u < kDecidePlanes; ++u) {
            const uint32_t b = 31u - (j0 + u);
            const uint32_t below = (b == 0u) ? 0u : ((1u << b) - 1u);
            // per-context all-ones / all-zero masks (uniform across the wave)
            uint32_t tsel[NC], nsel[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                tsel[i] = 0u - ((T[i] >> b) & 1u);
                nsel[i] = (T[i] & below) ? ~0u : 0u;
            }
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                uint32_t tb = 0u, nz = 0u;
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    tb |= cm[i][w] & tsel[i];
                    nz |= cm[i][w] & nsel[i];
                }
                lt[w] |= eq[w] & tb & ~R[u][w];
                eq[w] &= ~(tb ^ R[u][w]) & nz;
            }
        }
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) D[w] = lt[w];
}

// OR of v over the four lanes of a quad (DPP quad permutations).
__device__ __forceinline__ uint32_t quad_or(uint32_t v)
{
    v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
    return v | (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
}

// Transpose of a 4 x 4 word matrix held by a quad, row q in lane q: after
// it, R[x] of lane q is the old R[q] of lane x.  Two exchange steps: with
// lane q ^ 1 the words whose index differs from q in bit 0, then with lane
// q ^ 2 those that differ in bit 1.
__device__ __forceinline__ void quad_transpose(uint32_t (&R)[4], uint32_t q)
{
    const uint32_t odd1 = (q & 1u) ? ~0u : 0u, odd2 = (q & 2u) ? ~0u : 0u;
    uint32_t A[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const uint32_t other = (uint32_t)__builtin_amdgcn_mov_dpp((int)R[x ^ 1], 0xB1, 0xF, 0xF, false);
        const uint32_t keep = (x & 1) ? odd1 : ~odd1;   // index and lane agree in bit 0
        A[x] = (keep & R[x]) | (~keep & other);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const uint32_t other = (uint32_t)__builtin_amdgcn_mov_dpp((int)A[x ^ 2], 0x4E, 0xF, 0xF, false);
        const uint32_t keep = (x & 2) ? odd2 : ~odd2;   // ... in bit 1
        R[x] = (keep & A[x]) | (~keep & other);
    }
}

// The same decisions for a group held by the quad of lanes 4i .. 4i+3, lane
// q holding word q (sites 32q .. 32q+31) and calling this with the other
// three: in round m lane q draws plane 4m + q, the quad transposes the four
// draws so that each lane has its own word of the four planes, and each lane
// runs those planes in order over its 32 sites.  A site's decision is taken at
// its first plane whose bit differs from its threshold's or after which the
// threshold has no 1 bit left, as in the plane-by-plane loop; the quad stops
// when none of its sites is undecided.  D is this lane's word.
template <int NC>
__device__ __forceinline__ void decide32_quad(uint32_t key0, uint32_t key1, uint32_t g, uint32_t r, uint32_t t,
                                              uint32_t c, const uint32_t (&T)[NC], const uint32_t (&cm)[NC][1],
                                              const uint32_t (&live)[1], uint32_t q, uint32_t (&D)[1])
{
    // bit b of NZ[i]: T[i] has a 1 bit below bit b (bits above its lowest 1)
    uint32_t NZ[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const uint32_t low = T[i] & (0u - T[i]);
        NZ[i] = ~(low | (low - 1u));
    }
    uint32_t eq = live[0], lt = 0u;
    for (uint32_t j0 = 0; j0 < 32u; j0 += 4u) {
        if (quad_or(eq) == 0u) break;   // the same in the quad's four lanes
        uint32_t R[4];
        philox4x32_10(g, r, t, ((j0 + q) << 2) | c, key0, key1, R);
        quad_transpose(R, q);   // R[x]: this lane's word of plane j0 + x
        // the round's bits of each class: plane j0 + x compares bit 31 - x
        uint32_t Tr[NC], Nr[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            Tr[i] = T[i] << j0;
            Nr[i] = NZ[i] << j0;
        }
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            uint32_t tb = 0u, nz = 0u;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                tb |= cm[i][0] & (uint32_t)((int32_t)(Tr[i] << x) >> 31);
                nz |= cm[i][0] & (uint32_t)((int32_t)(Nr[i] << x) >> 31);
            }
            const uint32_t d = (tb ^ R[x]) | ~nz, l = tb & ~R[x];
            lt |= eq & l;
            eq &= ~d;
        }
    }
    D[0] = lt;
}

// Tile of work-group b of n in an XCD-aware order: work-groups are dispatched
// to the 8 XCDs in turn (b mod 8), and XCD x, which receives ceil((n - x) / 8)
// of them, takes the next contiguous range of tiles, so that neighbouring
// tiles, whose halos overlap, share that XCD's L2.  A permutation of 0..n-1.
// It suits tiles of equal work (each XCD gets a contiguous band of them).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n)
{
    const uint32_t x = b & 7u;
    uint32_t first = 0;
    for (uint32_t y = 0; y < x; ++y) first += (n + 7u - y) >> 3;
    return first + (b >> 3);
}

// Adds the per-cell quantity q of the calling thread to bin (X / B, Y / B).
// Launch shape: 16 x 16 threads per block over a 16 x 16 tile of cells.  When
// B is a multiple of 16 the whole tile falls in one bin and is reduced in the
// block first.
__device__ __forceinline__ void bin_add(uint64_t q, int X, int Y, bool valid, uint32_t B,
                                        uint32_t bins_x, unsigned long long *bin_sum)
{
    if ((B & 15u) == 0u) {
        __shared__ unsigned long long part[4];
        uint64_t v = valid ? q : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        const int tid = threadIdx.y * blockDim.x + threadIdx.x;
        if ((tid & 63) == 0) part[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            const uint64_t s = part[0] + part[1] + part[2] + part[3];
            const int X0 = blockIdx.x * 16, Y0 = blockIdx.y * 16;
            if (s) atomicAdd(&bin_sum[(size_t)(Y0 / B) * bins_x + X0 / B], (unsigned long long)s);
        }
    } else if (valid && q) {
        atomicAdd(&bin_sum[(size_t)(Y / (int)B) * bins_x + X / (int)B], (unsigned long long)q);
    }
}

}  // namespace tl
