// Measurement helper, not part of the sampler: the LDS read rate of gfx950
// with conflict-free 128-bit reads.  Every thread of 2048 blocks x 1024
// threads reads 16 bytes per iteration from a 64 KB LDS array (consecutive
// lanes read consecutive 16-byte words; the stride between iterations is a
// run-time argument, so no read can be folded away) and XOR/adds the values.
// Prints one JSON line: bytes read per launch, the best of five launch times
// and the rate.  Used to check, with rocprofv3 LDS counters, the LDS peak the
// sweep kernels are compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
            return 1;                                                              \
        }                                                                          \
    } while (0)

constexpr int kWords = 4096;   // uint4 words: 64 KB

__global__ void __launch_bounds__(1024) lds_read_kernel(uint32_t *out, int iters, int stride)
{
    __shared__ uint4 buf[kWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kWords; i += blockDim.x) buf[i] = make_uint4(i, 3u * i, 7u * i, 11u * i);
    __syncthreads();
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    int idx = tid & (kWords - 1);
    for (int k = 0; k < iters; ++k) {
        const uint4 v = buf[idx];
        acc.x ^= v.x;
        acc.y += v.y;
        acc.z ^= v.z;
        acc.w += v.w;
        idx = (idx + stride) & (kWords - 1);
    }
    // never true for these inputs; keeps the reads live
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9E3779B9u) out[(size_t)blockIdx.x * blockDim.x + tid] = acc.x;
}

int main(int argc, char **argv)
{
    const int stride = argc > 1 ? atoi(argv[1]) : 1024;
    const int blocks = 2048, threads = 1024, iters = 4096;
    uint32_t *out = nullptr;
    CHECK(hipMalloc(&out, (size_t)blocks * threads * sizeof(uint32_t)));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    float best = 1e30f;
    for (int rep = 0; rep < 5; ++rep) {
        CHECK(hipEventRecord(a, 0));
        hipLaunchKernelGGL(lds_read_kernel, dim3(blocks), dim3(threads), 0, 0, out, iters, stride);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(b, 0));
        CHECK(hipEventSynchronize(b));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, a, b));
        if (rep > 0 && ms < best) best = ms;
    }
    const double bytes = (double)blocks * threads * iters * 16.0;
    printf("{\"probe\": \"lds_read_b128\", \"stride_words\": %d, \"bytes_per_launch\": %.0f, \"best_ms\": %.4f, "
           "\"GB_per_s\": %.1f}\n", stride, bytes, best, bytes / (best * 1e-3) / 1e9);
    CHECK(hipFree(out));
    return 0;
}
