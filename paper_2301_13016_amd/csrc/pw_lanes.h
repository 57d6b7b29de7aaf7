// Cross-lane moves and fused multiply-adds shared by the kernels (device
// code): DPP shifts along the 64-lane wavefront, lane reads and fma in the
// compute type.
#pragma once

#include <hip/hip_runtime.h>

namespace pw {
namespace lanes {

// DPP controls (GFX9 family): wave_shr:1 moves lane l-1 into lane l,
// wave_shl:1 moves lane l+1 into lane l (bound_ctrl: the lane with no source
// reads 0).
constexpr int kWaveShr1 = 0x138;
constexpr int kWaveShl1 = 0x130;

template <int Ctrl> __device__ __forceinline__ float wave_shift(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), Ctrl, 0xf, 0xf, true));
}
template <int Ctrl> __device__ __forceinline__ double wave_shift(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), Ctrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), Ctrl, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double lane_value(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

template <typename T> __device__ __forceinline__ T fma_(T a, T b, T c);
template <> __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

}  // namespace lanes
}  // namespace pw
