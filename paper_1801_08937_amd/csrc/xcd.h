// Block-to-XCD mapping.  The hardware dispatches workgroups round-robin over
// the 8 XCDs (each with its own L2); xcd_block remaps the hardware block id so
// that each XCD works on a contiguous range of logical blocks, which then
// share their cache lines in that XCD's L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mm {

__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nb) {
    if ((nb & 7) != 0) return bid;
    return (bid & 7) * (nb >> 3) + (bid >> 3);
}

}  // namespace mm
