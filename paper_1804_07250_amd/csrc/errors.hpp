// Error reporting shared by the C-ABI translation units: tl::fail records a
// thread-local message (returned by tl_last_error) and returns the status.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/tilings.h"

#include <vector>

namespace tl {
tl_status fail(tl_status st, const char *fmt, ...);
// The HIP stream a sampler runs on.
hipStream_t sampler_stream(const tl_sampler *s);
// Threshold table of (domain, weights) as returned by tl_thresholds.
tl_status make_table(const tl_domain &d, const tl_weights &w, std::vector<uint32_t> &thr);
// Table of the free boundary points of a six-vertex mask (empty otherwise).
tl_status make_free_table(const tl_domain &d, const tl_weights &w, std::vector<uint32_t> &thr);
}

#define TL_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return tl::fail(TL_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                              \
    } while (0)
