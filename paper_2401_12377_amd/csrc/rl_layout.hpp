// Byte layout of one rigid-body RL scene arena (host and device).
#pragma once
#include <stdint.h>

#include "acs_tasks.h"

#if defined(__HIPCC__)
#define ACS_HD __host__ __device__
#else
#define ACS_HD
#endif

namespace acs {

constexpr int32_t kRLMaxBodies = 1024;

ACS_HD inline uint64_t rl_align(uint64_t x) { return (x + 255u) & ~uint64_t(255); }

// Offsets of the regions of enum acs_rl_region for n bodies.  The islands
// kernel's outputs (label .. padj) are contiguous so that one write range
// covers them; likewise deg .. adj for the broadphase kernel.
ACS_HD inline void rl_offsets(int32_t n, uint64_t *off)
{
    const uint64_t un = (uint64_t)n;
    const uint64_t vec = 16 * un, ints = 4 * un, ints1 = 4 * (un + 1), edges = 4 * un * (un - 1);
    const uint64_t sizes[ACS_RL_END] = {vec, vec, vec, vec, vec,
                                        ints, ints1, edges,
                                        ints, ints, ints, ints1,
                                        ints1, edges};
    uint64_t p = 0;
    for (int r = 0; r < ACS_RL_END; r++) {
        off[r] = p;
        p = rl_align(p + sizes[r]);
    }
    off[ACS_RL_END] = p;
}

// Entries of the host-visible plan buffer: 4 header ints + 4 per multi-body island.
ACS_HD inline uint64_t rl_plan_ints(int32_t n) { return 4 + 4 * (uint64_t)(n / 2); }

}  // namespace acs
