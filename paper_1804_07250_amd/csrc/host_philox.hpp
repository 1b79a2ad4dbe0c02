// Host-side Philox4x32-10 for the colour of each step under the random colour
// order (the one-launch-per-colour-step path picks its kernel on the host).
#pragma once
#include <stdint.h>

namespace tl {

// floor(K u / 2^32), u = word 0 of Philox4x32-10(key = (seed mod 2^32,
// seed >> 32), ctr = (step, 0, 0, 2^31)).
uint32_t host_step_colour(uint64_t seed, uint32_t step, uint32_t K);

}  // namespace tl
