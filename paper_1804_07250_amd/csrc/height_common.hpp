// Shared pieces of the two height-function models (lozenge, six-vertex):
// plane layout helpers, shifted word reads, per-row site masks.
//
// Layout: plane p, row y, word w at planes[p*PS + y*RS + 4 + w].  Each row
// starts and ends with a zero pad group of 4 words, so reads at w-1 and w+4
// of a group stay inside the row.  RS = 4*(ng + 2).
#pragma once
#include "device_common.hpp"

namespace tl {

__device__ __forceinline__ void hld4(const uint32_t *p, uint32_t (&v)[4])
{
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
}
__device__ __forceinline__ void hst4(uint32_t *p, const uint32_t (&v)[4])
{
    *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
}

// Words 4g..4g+3 of a plane row, as seen by a site one position to the
// right (+1: site k reads bit k+1) or left (-1: site k reads bit k-1).
// p points at word 4g; p[-1] and p[4] exist (pad groups).
__device__ __forceinline__ void hld4_plus1(const uint32_t *p, uint32_t (&v)[4])
{
    uint32_t a[4];
    hld4(p, a);
    const uint32_t nxt = p[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) v[w] = (a[w] >> 1) | (((w < 3) ? a[w + 1] : nxt) << 31);
}
__device__ __forceinline__ void hld4_minus1(const uint32_t *p, uint32_t (&v)[4])
{
    uint32_t a[4];
    hld4(p, a);
    const uint32_t prv = p[-1];
#pragma unroll
    for (int w = 0; w < 4; ++w) v[w] = (a[w] << 1) | (((w > 0) ? a[w - 1] : prv) >> 31);
}

// Bits of word w (sites k = 32w .. 32w+31) with klo <= k <= khi.
__device__ __forceinline__ uint32_t range_mask(int w, int klo, int khi)
{
    const int lo = klo - 32 * w, hi = khi - 32 * w;
    if (hi < 0 || lo > 31 || hi < lo) return 0u;
    const int l = lo < 0 ? 0 : lo, h = hi > 31 ? 31 : hi;
    const uint32_t up = (h == 31) ? 0xFFFFFFFFu : ((1u << (h + 1)) - 1u);
    return up & ~((1u << l) - 1u);
}

// floor(a / b) for b > 0.
__device__ __forceinline__ int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

}  // namespace tl
