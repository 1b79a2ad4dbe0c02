// Reference Philox4x32-10 outputs from rocRAND's engine (host path of the
// header-only implementation).  Reads "k0 k1 c0 c1 c2 c3" lines from stdin and
// prints the four output words of Philox(ctr=(c0,c1,c2,c3), key=(k0,k1)).
// Counter mapping of the engine: key = seed, counter.zw = subsequence,
// counter.xy = offset / 4.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = 4ULL * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
