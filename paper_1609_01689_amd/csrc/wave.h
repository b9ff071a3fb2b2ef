// Wavefront-level helpers for doubles (64-lane waves of gfx950): DPP lane
// moves, lane reads and butterfly sums that stay out of LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace hsym {

// Cross-lane moves of a double through DPP (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
// Sums over a quad / a row of 16 lanes / the wave.  Every lane receives the
// bitwise identical sum (each butterfly step adds the same two operands, in
// either order).  Called with the whole wave active.
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    return v;
}
__device__ __forceinline__ double row_sum(double v) {
    v = quad_sum(v);
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    v = row_sum(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

}  // namespace hsym
