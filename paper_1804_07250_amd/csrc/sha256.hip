// SHA-256 (FIPS 180-4) for the canonical hash: one device thread hashes one row
// of the canonical export; the host hashes the concatenated row digests.
// The round constants are derived from their definition (first 32 bits of the
// fractional parts of the cube roots of the first 64 primes; the initial hash
// value from the square roots of the first 8 primes).
#include <math.h>
#include <string.h>

#include "internal.hpp"

namespace tl {

namespace {

struct ShaConst {
    uint32_t k[64];
    uint32_t h0[8];
};

uint32_t frac32(long double v)
{
    long double f = v - floorl(v);
    return (uint32_t)floorl(ldexpl(f, 32));
}

ShaConst make_consts()
{
    ShaConst c;
    int primes[64], np = 0;
    for (int p = 2; np < 64; ++p) {
        bool prime = true;
        for (int q = 2; q * q <= p; ++q)
            if (p % q == 0) {
                prime = false;
                break;
            }
        if (prime) primes[np++] = p;
    }
    for (int i = 0; i < 64; ++i) {
        // cube root refined by Newton steps in extended precision
        long double x = cbrtl((long double)primes[i]);
        for (int it = 0; it < 3; ++it) x = x - (x * x * x - primes[i]) / (3 * x * x);
        c.k[i] = frac32(x);
    }
    for (int i = 0; i < 8; ++i) c.h0[i] = frac32(sqrtl((long double)primes[i]));
    return c;
}

const ShaConst &consts()
{
    static const ShaConst c = make_consts();
    return c;
}

__host__ __device__ inline uint32_t rotr(uint32_t x, int s) { return (x >> s) | (x << (32 - s)); }

// One compression: the message schedule kept as a rolling window of 16 words
// (w[i & 15] holds W_i once round i needs it), fully unrolled, so that on the
// device every word stays in a register.
__host__ __device__ inline void compress(uint32_t st[8], const uint32_t m[16], const uint32_t *K)
{
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = m[i];
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3], e = st[4], f = st[5], g = st[6], h = st[7];
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        if (i >= 16) {
            const uint32_t x = w[(i - 15) & 15], y = w[(i - 2) & 15];
            const uint32_t s0 = rotr(x, 7) ^ rotr(x, 18) ^ (x >> 3);
            const uint32_t s1 = rotr(y, 17) ^ rotr(y, 19) ^ (y >> 10);
            w[i & 15] += s0 + w[(i - 7) & 15] + s1;
        }
        const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
        const uint32_t ch = (e & f) ^ (~e & g);
        const uint32_t t1 = h + S1 + ch + K[i] + w[i & 15];
        const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
        const uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
        const uint32_t t2 = S0 + mj;
        h = g;
        g = f;
        f = e;
        e = d + t1;
        d = c;
        c = b;
        b = a;
        a = t1 + t2;
    }
    st[0] += a;
    st[1] += b;
    st[2] += c;
    st[3] += d;
    st[4] += e;
    st[5] += f;
    st[6] += g;
    st[7] += h;
}

// Byte i of the padded message (data, len bytes; total padded length plen).
__host__ __device__ inline uint8_t padded_byte(const uint8_t *data, uint64_t len, uint64_t plen, uint64_t i)
{
    if (i < len) return data[i];
    if (i == len) return 0x80u;
    if (i >= plen - 8) {
        const uint64_t bits = len * 8ull;
        return (uint8_t)(bits >> (8 * (plen - 1 - i)));
    }
    return 0u;
}

__host__ __device__ inline void sha256_any(const uint8_t *data, uint64_t len, const uint32_t *K,
                                           const uint32_t *H0, uint8_t out[32])
{
    uint32_t st[8];
    for (int i = 0; i < 8; ++i) st[i] = H0[i];
    const uint64_t plen = ((len + 8) / 64 + 1) * 64;
    // whole blocks of a 16-byte aligned message are read a word at a time
    const bool aligned = ((uintptr_t)data & 15u) == 0u;
    for (uint64_t blk = 0; blk < plen; blk += 64) {
        uint32_t m[16];
        if (blk + 64 <= len && aligned) {
            const uint32_t *p = reinterpret_cast<const uint32_t *>(data + blk);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t v = p[i];   // bytes of a little-endian word, read big-endian
                m[i] = (v >> 24) | ((v >> 8) & 0xFF00u) | ((v << 8) & 0xFF0000u) | (v << 24);
            }
        } else if (blk + 64 <= len) {
            for (int i = 0; i < 16; ++i) {
                const uint8_t *p = data + blk + 4 * i;
                m[i] = ((uint32_t)p[0] << 24) | ((uint32_t)p[1] << 16) | ((uint32_t)p[2] << 8) | p[3];
            }
        } else {
            for (int i = 0; i < 16; ++i) {
                uint32_t v = 0;
                for (int j = 0; j < 4; ++j) v = (v << 8) | padded_byte(data, len, plen, blk + 4 * i + j);
                m[i] = v;
            }
        }
        compress(st, m, K);
    }
    for (int i = 0; i < 8; ++i) {
        out[4 * i] = (uint8_t)(st[i] >> 24);
        out[4 * i + 1] = (uint8_t)(st[i] >> 16);
        out[4 * i + 2] = (uint8_t)(st[i] >> 8);
        out[4 * i + 3] = (uint8_t)st[i];
    }
}

struct ShaArgs {
    uint32_t k[64];
    uint32_t h0[8];
};

__global__ void hash_rows_kernel(const uint8_t *data, uint32_t rows, uint32_t row_bytes, uint8_t *digests,
                                 ShaArgs c)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    sha256_any(data + (size_t)r * row_bytes, row_bytes, c.k, c.h0, digests + 32 * (size_t)r);
}

}  // namespace

void sha256_host(const uint8_t *data, size_t len, uint8_t out[32])
{
    const ShaConst &c = consts();
    sha256_any(data, len, c.k, c.h0, out);
}

hipError_t hash_rows(const uint8_t *data, uint32_t rows, uint32_t row_bytes, uint8_t *digests, hipStream_t s)
{
    const ShaConst &c = consts();
    ShaArgs a;
    memcpy(a.k, c.k, sizeof a.k);
    memcpy(a.h0, c.h0, sizeof a.h0);
    dim3 block(64), grid((rows + 63) / 64);
    hipLaunchKernelGGL(hash_rows_kernel, grid, block, 0, s, data, rows, row_bytes, digests, a);
    return hipGetLastError();
}

}  // namespace tl
