// Fixed-order FP64 sum over the 64 lanes of a wavefront (device code), shared
// by the kernels that reduce per-wavefront partials: the same value in every
// lane and the same order on every run.
#pragma once

#include <hip/hip_runtime.h>

#include "pw_lanes.h"

namespace pw {
namespace red {

// x moved across lanes by a DPP control that gives every lane a source (a
// permutation within quads or rows), both halves of the double.
template <int Ctrl> __device__ __forceinline__ double dpp_move(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), Ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), Ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowRor4 = 0x124;   // rotate by 4 within a row of 16 lanes
constexpr int kRowRor8 = 0x128;   // rotate by 8

using lanes::lane_value;

// Pairs and quads (quad permutations), the four quads of each 16-lane row
// (row rotations), then the four row sums in a fixed order.  All register
// moves (DPP, readlane): no LDS traffic and no waits.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_move<kQuadXor1>(x);
    x += dpp_move<kQuadXor2>(x);
    x += dpp_move<kRowRor4>(x);
    x += dpp_move<kRowRor8>(x);
    return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}

}  // namespace red
}  // namespace pw
