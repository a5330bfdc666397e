// Cross-lane moves inside one 64-lane wavefront, by DPP wavefront shifts
// (v_mov_b32_dpp wave_shr:1 / wave_shl:1, a register-to-register move with
// no LDS traffic).
//   lane_from_left(x)  returns x of lane - 1 (lane 0 keeps its own value)
//   lane_from_right(x) returns x of lane + 1 (lane 63 keeps its own value)
// The edge lanes are halo lanes in every caller; their results are unused.
// Every lane of the wavefront must execute the call.
#pragma once
#include <hip/hip_runtime.h>

namespace elwh {

__device__ __forceinline__ int dpp_from_left_i(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_from_right_i(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x130, 0xf, 0xf, false); }

__device__ __forceinline__ float lane_from_left(float x) { return __int_as_float(dpp_from_left_i(__float_as_int(x))); }
__device__ __forceinline__ float lane_from_right(float x) { return __int_as_float(dpp_from_right_i(__float_as_int(x))); }

__device__ __forceinline__ double lane_from_left(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_from_left_i((int)(b & 0xffffffffLL));
    const int hi = dpp_from_left_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_from_right_i((int)(b & 0xffffffffLL));
    const int hi = dpp_from_right_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The same shifts with the edge lane's result undefined in effect (it reads
// 0): the move has no "old" operand, so the compiler may fold it into the
// instruction that consumes it (a DPP source operand) instead of copying the
// register first.  For callers whose edge lanes are never used.
__device__ __forceinline__ float lane_from_left_z(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right_z(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_from_left_z(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right_z(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace elwh
