// Inputs for the autotuner's timing runs.  Kernel times depend on the data
// as well as the shape (the same forward runs 2-3 % faster on zeros than on
// winds of the workload's scale, and not by the same amount for every shape),
// so shapes are ranked on values like the ones they will meet: uniform in
// [lo, hi), from a counter-based hash of the element index, stored in the
// array's type.  These values only feed timings; nothing is checked against
// them.
#include <algorithm>

#include "pw_internal.h"

namespace pw {
namespace {

// The 32-bit finalizer of MurmurHash3 (fmix32): a bijective mix in which
// every input bit affects every output bit.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

template <typename T> __device__ __forceinline__ T store_as(float x);
template <> __device__ __forceinline__ float store_as<float>(float x) { return x; }
template <> __device__ __forceinline__ double store_as<double>(float x) { return static_cast<double>(x); }
template <> __device__ __forceinline__ uint16_t store_as<uint16_t>(float x) {   // BF16: upper half (truncated)
    return static_cast<uint16_t>(__float_as_uint(x) >> 16);
}
template <> __device__ __forceinline__ _Float16 store_as<_Float16>(float x) { return static_cast<_Float16>(x); }

template <typename T>
__global__ void tune_fill_kernel(T *p, int64_t n, uint32_t seed, float lo, float span) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t h = fmix32(static_cast<uint32_t>(i) ^ fmix32(static_cast<uint32_t>(i >> 32) + seed));
        const float u = static_cast<float>(h >> 8) * (1.0f / 16777216.0f);   // [0, 1)
        p[i] = store_as<T>(lo + span * u);
    }
}

template <typename T> hipError_t fill_t(void *p, int64_t n, uint32_t seed, float lo, float hi, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(tune_fill_kernel<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, static_cast<T *>(p), n,
                       seed, lo, hi - lo);
    return hipGetLastError();
}

}  // namespace

hipError_t fill_tuning_data(void *p, int64_t n, pw_dtype dt, uint32_t seed, float lo, float hi, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (dt) {
        case PW_F32: return fill_t<float>(p, n, seed, lo, hi, s);
        case PW_F64: return fill_t<double>(p, n, seed, lo, hi, s);
        case PW_BF16: return fill_t<uint16_t>(p, n, seed, lo, hi, s);
        case PW_F16: return fill_t<_Float16>(p, n, seed, lo, hi, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace pw
