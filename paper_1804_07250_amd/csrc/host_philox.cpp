// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) on the host: ten rounds of
// two 32 x 32 -> 64-bit products with the key bumped by the Weyl constants.
#include "host_philox.hpp"

namespace tl {

uint32_t host_step_colour(uint64_t seed, uint32_t step, uint32_t K)
{
    uint32_t c[4] = {step, 0u, 0u, 0x80000000u};
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
    }
    return (uint32_t)(((uint64_t)c[0] * K) >> 32);
}

}  // namespace tl
