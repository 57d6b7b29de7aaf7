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

// Six FP64 values per lane, each summed over the wavefront, with the work
// shared out instead of six separate sums (about 60 instead of 140
// instructions).  The six are padded to eight; at each butterfly step a lane
// keeps half of its values and adds its partner's copy of them, sending the
// other half: pairs (lane ^ 1) split 8 into 4, pairs (lane ^ 2) 4 into 2,
// lanes four apart within a 16-lane row 2 into 1.  Then every lane holds one
// quantity, q(l) = 4 (l & 1) + 2 ((l >> 1) & 1) + ((l >> 2) & 1), summed over
// 8 lanes, which lanes eight apart in the row, then 16 and 32 apart in the
// wavefront add up.  Returns in every lane the total of its quantity q(l)
// (6 and 7: zero).  The order of every addition is fixed, so the result is
// the same on every run.
__device__ __forceinline__ int sum6_quantity(int lane) {
    return 4 * (lane & 1) + 2 * ((lane >> 1) & 1) + ((lane >> 2) & 1);
}
__device__ __forceinline__ double bpermute_from(double x, int src_lane) {
    const int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, __double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum6(const double (&q)[6]) {
    const int lane = static_cast<int>(threadIdx.x & 63);
    const bool b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1;
    const double v[8] = {q[0], q[1], q[2], q[3], q[4], q[5], 0.0, 0.0};
    double k4[4], k2[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {   // keep quantities 4 b0 + j
        const double send = b0 ? v[j] : v[4 + j];
        k4[j] = (b0 ? v[4 + j] : v[j]) + dpp_move<kQuadXor1>(send);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {   // keep 4 b0 + 2 b1 + j
        const double send = b1 ? k4[j] : k4[2 + j];
        k2[j] = (b1 ? k4[2 + j] : k4[j]) + dpp_move<kQuadXor2>(send);
    }
    // the lane four places away in the row has the other b2: it sends what this lane keeps
    double t = (b2 ? k2[1] : k2[0]) + dpp_move<kRowRor4>(b2 ? k2[0] : k2[1]);
    t += dpp_move<kRowRor8>(t);
    t += bpermute_from(t, lane ^ 16);
    t += bpermute_from(t, lane ^ 32);
    return t;
}

}  // namespace red
}  // namespace pw
