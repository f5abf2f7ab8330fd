// Workgroup renumbering for the 8 XCDs of the MI355X. Workgroups are dispatched round-robin
// over the XCDs (workgroup b runs on XCD b mod 8), each with its own L2. xcd_block() maps them
// so that every XCD processes one contiguous range of the grid's blocks: neighbouring rows (or
// node tiles) gather neighbouring vector entries (or feature rows), which then stay in one L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgg {

__device__ __forceinline__ int32_t xcd_block() {
    constexpr int32_t kXcd = 8;
    const int32_t b = blockIdx.x, g = gridDim.x;
    const int32_t q = g / kXcd, r = g % kXcd;
    const int32_t x = b % kXcd, k = b / kXcd;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

}  // namespace amgg
