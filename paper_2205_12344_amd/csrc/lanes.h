// Cross-lane moves inside one 64-lane wavefront.
//   lane_from_left(x)  returns x of lane - 1 (lane 0 gets its own value)
//   lane_from_right(x) returns x of lane + 1 (lane 63 gets its own value)
// The edge lanes are halo lanes in every caller; their results are unused.
#pragma once
#include <hip/hip_runtime.h>

namespace elwh {

__device__ __forceinline__ float lane_from_left(float x) { return __shfl_up(x, 1, 64); }
__device__ __forceinline__ float lane_from_right(float x) { return __shfl_down(x, 1, 64); }
__device__ __forceinline__ double lane_from_left(double x) { return __shfl_up(x, 1, 64); }
__device__ __forceinline__ double lane_from_right(double x) { return __shfl_down(x, 1, 64); }

}  // namespace elwh
