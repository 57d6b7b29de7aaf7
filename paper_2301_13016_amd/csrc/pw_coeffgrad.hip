// Gradients of L = <su, gsu> + <sv, gsv> + <sw, gsw> with respect to the
// coefficients, gfx950.  L is linear in every coefficient: each term of the
// operator is one coefficient times a coefficient-free product, so dL/dc sums,
// over the terms c multiplies, the cotangent at the term's output point times
// that product.  tcx and tcy multiply the x- and y-face terms at every point;
// tzc1[k], tzc2[k] (u, v) and tzd1[k], tzd2[k] (w) the lower / upper z-face
// terms of level k.
//
// Pass 1 is the adjoint kernel's march (pw_adjoint.hip, cg_level), alone or
// together with the wind gradients: every wavefront evaluates the six
// coefficient-free term groups at its points, weights them by the
// cotangents, sums per lane and then across the wavefront in FP64, and writes
// one partial per (quantity, level, strip) to the workspace.  Pass 2 (here)
// sums the strips of each (quantity, level) in a fixed order, and pass 3 the
// levels of tcx and tcy.  No atomics: the result is the same on every run,
// and the same whether or not the wind gradients were computed in pass 1.
#include <mutex>

#include "pw_internal.h"
#include "pw_reduce.h"

namespace pw {
namespace {

constexpr int kQ = 6;   // tzc1, tzc2, tzd1, tzd2, tcx (level share), tcy (level share)

// Pass 2: out[q*nz + k] = sum over strips of ws[q][k][strip], one workgroup
// per (q, k), a fixed order (strided per thread, then a tree in LDS).
__global__ __launch_bounds__(256) void pw_coeffgrad_reduce_kernel(const double *__restrict__ ws, int64_t nstrips,
                                                                  double *__restrict__ out) {
    __shared__ double part[256];
    const double *row = ws + static_cast<int64_t>(blockIdx.x) * nstrips;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nstrips; i += 256) s += row[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// Pass 3: out[6*nz + q] = sum over levels of the tcx (q = 0) / tcy (q = 1)
// level shares; wavefront q adds lane-strided levels, then a butterfly (a
// fixed order).
__global__ __launch_bounds__(128) void pw_coeffgrad_total_kernel(double *__restrict__ out, int nz) {
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double *lv = out + (4 + q) * nz;
    double s = 0.0;
    for (int k = lane; k < nz; k += 64) s += lv[k];
    s = red::wave_sum(s);
    if (lane == 0) out[6 * nz + q] = s;
}

// Scratch of the allocation-free entry point (pw_advect_coeff_grad_static):
// the per-strip partials of one call live in this array instead of a caller
// workspace.  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never uses the array's name as an address (on the
// host it is a stand-in, not device memory); it uses the address that
// hipGetSymbolAddress returns on each device.
static __device__ __align__(256) double scratch[kCoeffGradScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

}  // namespace

pw_status coeff_grad_scratch(void **ptr) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PW_ERR_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e2 = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e2 != hipSuccess) return hip_fail(e2, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PW_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PW_OK;
}

int64_t coeff_grad_workspace_bytes(const pw_grid &g, pw_dtype dt) {
    (void)dt;
    // partials of the adjoint's strips, for any rows per strip (one row: the most strips)
    return kQ * g.nz * adjoint_strips(g, 1) * static_cast<int64_t>(sizeof(double));
}

pw_status launch_coeff_grad_reduce(const double *partials, int64_t nstrips, double *grad, int64_t nz,
                                   hipStream_t s) {
    if (nstrips <= 0 || nstrips > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    hipLaunchKernelGGL(pw_coeffgrad_reduce_kernel, dim3(static_cast<unsigned>(kQ * nz)), dim3(256), 0, s, partials,
                       nstrips, grad);
    const pw_status st = hip_fail(hipGetLastError(), "coefficient gradient reduction launch");
    if (st != PW_OK) return st;
    hipLaunchKernelGGL(pw_coeffgrad_total_kernel, dim3(1), dim3(128), 0, s, grad, static_cast<int>(nz));
    return hip_fail(hipGetLastError(), "coefficient gradient total launch");
}

}  // namespace pw
