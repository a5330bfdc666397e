// XCD-aware workgroup-to-tile mapping for the stencil kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace elwh {

// XCD-banded tile order.  The workgroups of a launch are dealt round-robin
// to the eight XCDs, each with its own L2; workgroup b is given tile
// t = (b mod 8) * ceil(ntiles / 8) + b / 8, so every XCD works through one
// contiguous band of tiles (row-major over x-strip, row chunk) and the halo
// rows and columns that neighbouring tiles share are read through the same
// L2 instead of twice from the fabric.  The grid is 8 ceil(ntiles / 8)
// workgroups; false for the padding workgroups.
constexpr int kXcds = 8;

__host__ __device__ __forceinline__ int xcd_grid(int ntiles) { return kXcds * ((ntiles + kXcds - 1) / kXcds); }

__device__ __forceinline__ bool xcd_tile(int b, int ntiles, int& t) {
    const int per = (ntiles + kXcds - 1) / kXcds;
    t = (b % kXcds) * per + b / kXcds;
    return t < ntiles;
}

}  // namespace elwh
