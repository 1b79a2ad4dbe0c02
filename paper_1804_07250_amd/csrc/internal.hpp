// Host-side interfaces between the C-ABI layer (api.hip) and the per-model
// kernel launchers.  Every launcher enqueues on the given stream and returns the
// HIP status of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tl {

// Threshold values handed to a colour-step kernel by value.
struct Thr {
    uint32_t v[32];
};

// ---------------------------------------------------------------- domino
// Aztec diamond of order n in the owner frame: the owner colour
// omega = (n+1) mod 2 has its n^2 sites on the grid (r, k) in [0, n)^2; each
// owner site keeps the four crossing bits of its edges N, S, E, W (so every edge
// of the lattice is stored once, 4 bits per owner vertex = 2 bits per face).
// Plane p (N=0, S=1, E=2, W=3) row r word w lives at planes[p*PS + r*RS + w].
// RS = 4*(ng+1) words (ng groups of 4 words cover the row, 4 zero pad words),
// n+1 rows (row n is zero padding).
struct DominoDev {
    int n = 0;
    int omega = 0;
    uint32_t ng = 0;   // groups of 128 sites per row
    uint32_t RS = 0;   // row stride in words
    size_t PS = 0;     // plane stride in words
    uint32_t *planes = nullptr;
};
size_t domino_words(int n, uint32_t *ng, uint32_t *RS, size_t *PS);
hipError_t domino_init(const DominoDev &d, int init_max, hipStream_t s);
hipError_t domino_colour_step(const DominoDev &d, int colour, uint32_t t, const Thr &T, int metropolis,
                              uint64_t seed, hipStream_t s);
hipError_t domino_export(const DominoDev &d, uint8_t *faces, hipStream_t s);
hipError_t domino_observe(const DominoDev &d, uint32_t B, uint32_t bins_x, unsigned long long *bins,
                          hipStream_t s);

// ----------------------------------------------------------------- hashing
// SHA-256 of each of `rows` rows of `row_bytes` bytes at `data` (device), into
// 32-byte digests at `digests` (device).
hipError_t hash_rows(const uint8_t *data, uint32_t rows, uint32_t row_bytes, uint8_t *digests,
                     hipStream_t s);
void sha256_host(const uint8_t *data, size_t len, uint8_t out[32]);

}  // namespace tl
