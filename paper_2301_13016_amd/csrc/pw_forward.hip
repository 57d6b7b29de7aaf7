// Forward Piacsek-Williams advection kernel for gfx950 (CDNA4).
//
// What it computes: the source terms su, sv, sw of the PW scheme (paper
// Sec. 2.2; per-cell arithmetic of Sec. 4 / Fig. 2: six face sums, six
// products with a neighbouring value, signed reduction, same arithmetic for
// the three fields).  The equations are written out in include/pwadv.h.
//
// How (one wavefront = one independent work item, no LDS, no barriers):
//   * A wavefront owns a strip of 64*PX output columns x RY output rows and
//     marches upward through a chunk of z-levels.  Lane l owns PX consecutive
//     columns, loaded as one vector (unaligned vector loads are legal on this
//     target) and stored as one vector, so a row of the strip is one
//     contiguous 256*PX-byte (FP32) access per wavefront instruction and
//     output rows are written in whole, aligned pieces.
//   * x-neighbours: inside a lane they are register neighbours; across lanes
//     they come from DPP wavefront shifts of the first / last component; the
//     two columns outside the strip (left of lane 0, right of lane 63) come
//     from one extra "halo" load per plane and field in which lane r fetches
//     the left halo of row r and lane 32+r the right one, broadcast with
//     readlane.
//   * Each lane keeps RY+2 rows (the strip plus one halo row above and below)
//     of u, v, w for four consecutive z-planes in registers: planes k-1, k,
//     k+1 feed the stencil at level k while plane k+2 is in flight.  The ring
//     is rotated by unrolling the march four ways, so no register moves.
//   * Workgroups are re-numbered so that each XCD (8 per MI355X, each with its
//     own L2) gets one contiguous range of tiles, ordered z-chunk fastest:
//     tiles that share halo planes and rows run on the same L2.
//
// Storage types: float, double, BF16 (uint16_t bit patterns) and FP16
// (_Float16).  16-bit values are widened exactly to float as they arrive;
// the arithmetic is float (double for double storage), with explicit fma and
// a fixed order per point, so results do not depend on the launch shape.
#include "pw_stencil.h"

namespace pw {
namespace {

using namespace dev;

// Depth: planes in flight ahead of the level being computed (1 or 2).
// MaxT: the workgroup size bound the kernel is compiled for.  Every shape is
// built twice: for up to 256 threads (four wavefronts, one per SIMD, so a
// wavefront may use the whole 512-entry register file: the large strips keep
// their planes in registers instead of spilling) and for up to 512.
template <typename Tin, int PX, int RY, int Depth, int MaxT>
__global__ __launch_bounds__(MaxT) void pw_forward_kernel(FwdK<Tin> a) {
    // wavefront index as a scalar, so that per-strip conditions stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cz = t % a.nzc;
    const int t2 = t / a.nzc;
    const int tx = t2 % a.ntx;
    const int ty = (t2 / a.ntx) * a.wpb + wave;
    if (ty >= a.nty) return;   // whole wavefront
    strip_march<Tin, PX, RY, Depth>(a, tx, ty, cz);
}

template <typename Tin, int PX, int RY>
pw_status launch_fwd_t(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    using Tc = typename Storage<Tin>::Tc;
    FwdK<Tin> a;
    a.u = static_cast<const Tin *>(g.u);
    a.v = static_cast<const Tin *>(g.v);
    a.w = static_cast<const Tin *>(g.w);
    a.su = static_cast<Tc *>(g.su);
    a.sv = static_cast<Tc *>(g.sv);
    a.sw = static_cast<Tc *>(g.sw);
    a.tzc1 = static_cast<const Tc *>(g.tzc1);
    a.tzc2 = static_cast<const Tc *>(g.tzc2);
    a.tzd1 = static_cast<const Tc *>(g.tzd1);
    a.tzd2 = static_cast<const Tc *>(g.tzd2);
    a.tcx = static_cast<Tc>(g.tcx);
    a.tcy = static_cast<Tc>(g.tcy);
    a.nx = static_cast<int32_t>(g.nx);
    a.ny = static_cast<int32_t>(g.ny);
    a.nz = static_cast<int32_t>(g.nz);
    a.h = g.h;
    a.in_sz = g.in_sz;
    a.out_sz = g.out_sz;
    a.in_sy = static_cast<int32_t>(g.in_sy);
    a.out_sy = static_cast<int32_t>(g.out_sy);
    a.ntx = static_cast<int32_t>((g.nx + 64 * PX - 1) / (64 * PX));
    a.nty = static_cast<int32_t>((g.ny + RY - 1) / RY);
    a.zlen = cfg.zlen;
    a.nzc = static_cast<int32_t>((g.nz + cfg.zlen - 1) / cfg.zlen);
    a.wpb = cfg.wpb;
    const int64_t nblk_y = (a.nty + cfg.wpb - 1) / cfg.wpb;
    const int64_t nblocks = static_cast<int64_t>(a.ntx) * nblk_y * a.nzc;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    const dim3 grid(static_cast<unsigned>(nblocks)), block(64 * cfg.wpb);
    if (cfg.depth == 2) {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 2, 256>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 2, 512>), grid, block, 0, s, a);
    } else {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 1, 256>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 1, 512>), grid, block, 0, s, a);
    }
    return hip_fail(hipGetLastError(), "forward kernel launch");
}

template <typename Tin, int PX>
pw_status launch_fwd_px(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.ry) {
        case 1: return launch_fwd_t<Tin, PX, 1>(g, cfg, s);
        case 2: return launch_fwd_t<Tin, PX, 2>(g, cfg, s);
        case 4:
            if constexpr ((sizeof(Tin) <= 4 && PX <= 2) || (sizeof(Tin) == 2 && PX == 4))
                return launch_fwd_t<Tin, PX, 4>(g, cfg, s);
            [[fallthrough]];
        default:
            return fail(PW_ERR_UNSUPPORTED, "rows per strip %d with %d columns per lane not instantiated", cfg.ry,
                        PX);
    }
}

template <typename Tin>
pw_status launch_fwd_dt(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.px) {
        case 1: return launch_fwd_px<Tin, 1>(g, cfg, s);
        case 2: return launch_fwd_px<Tin, 2>(g, cfg, s);
        case 4:
            if constexpr (sizeof(Tin) <= 4) return launch_fwd_px<Tin, 4>(g, cfg, s);
            return fail(PW_ERR_UNSUPPORTED, "4 columns per lane not instantiated for this dtype");
        case 8:
            if constexpr (sizeof(Tin) == 2) return launch_fwd_px<Tin, 8>(g, cfg, s);
            [[fallthrough]];
        default: return fail(PW_ERR_UNSUPPORTED, "%d columns per lane not instantiated", cfg.px);
    }
}

// Plain device copy, 16 bytes per lane per step, grid-stride.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy16_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                     int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        u32x4 x = __builtin_nontemporal_load(src + i);
        __builtin_nontemporal_store(x, dst + i);
    }
}

// Three copies in one grid-stride loop: the stencil's traffic pattern (three
// arrays read, three written) without the stencil.
__global__ __launch_bounds__(256) void copy16x3_kernel(const u32x4 *__restrict__ a, const u32x4 *__restrict__ b,
                                                       const u32x4 *__restrict__ c, u32x4 *__restrict__ x,
                                                       u32x4 *__restrict__ y, u32x4 *__restrict__ z, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const u32x4 p = __builtin_nontemporal_load(a + i);
        const u32x4 q = __builtin_nontemporal_load(b + i);
        const u32x4 r = __builtin_nontemporal_load(c + i);
        __builtin_nontemporal_store(p, x + i);
        __builtin_nontemporal_store(q, y + i);
        __builtin_nontemporal_store(r, z + i);
    }
}

}  // namespace

bool tile_supported(const TileCfg &c, pw_dtype dt) {
    if (c.zlen < 1 || c.wpb < 1 || c.wpb > 8 || (c.depth != 1 && c.depth != 2)) return false;
    const bool half = dt == PW_BF16 || dt == PW_F16;
    if (dt == PW_F64) return (c.px == 1 || c.px == 2) && (c.ry == 1 || c.ry == 2);
    if (c.px == 8) return half && (c.ry == 1 || c.ry == 2);
    if (c.px == 4) return c.ry == 1 || c.ry == 2 || (half && c.ry == 4);
    return (c.px == 1 || c.px == 2) && (c.ry == 1 || c.ry == 2 || c.ry == 4);
}

TileCfg default_forward_tile(const FwdArgs &a, pw_dtype dt) {
    // Measured on MI355X (512x512x64 and 1024x1024x256): four columns per lane
    // in one-row strips for FP32, two columns in two-row strips for 16-bit
    // storage, one column in two-row strips for FP64 (register budget); four
    // strips per workgroup; the march cut into at least two z-chunks, more
    // when the grid has too few strips for about 8 wavefronts per CU.
    TileCfg c;
    c.wpb = 4;
    if (dt == PW_F32) {
        c.px = 4;
        c.ry = 1;
    } else if (dt == PW_F64) {
        c.px = 1;
        c.ry = 2;
    } else {
        c.px = 2;
        c.ry = 2;
    }
    const int64_t strips = ((a.nx + 64 * c.px - 1) / (64 * c.px)) * ((a.ny + c.ry - 1) / c.ry);
    int64_t chunks = (2048 + strips - 1) / strips;
    if (chunks < 2) chunks = 2;
    int64_t zl = (a.nz + chunks - 1) / chunks;
    if (zl < 8) zl = 8;
    if (zl > a.nz) zl = a.nz;
    c.zlen = static_cast<int>(zl);
    return c;
}

pw_status launch_forward(const FwdArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s) {
    if (!tile_supported(cfg, dt)) return fail(PW_ERR_INVALID_ARG, "unsupported tile configuration");
    switch (dt) {
        case PW_F32: return launch_fwd_dt<float>(a, cfg, s);
        case PW_F64: return launch_fwd_dt<double>(a, cfg, s);
        case PW_BF16: return launch_fwd_dt<uint16_t>(a, cfg, s);
        case PW_F16: return launch_fwd_dt<_Float16>(a, cfg, s);
    }
    return fail(PW_ERR_UNSUPPORTED, "dtype %d", static_cast<int>(dt));
}

pw_status launch_copy3(const void *const *src, void *const *dst, int64_t nbytes, hipStream_t s) {
    const int64_t n = nbytes / 16;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;   // measured best for this pattern on MI355X
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(copy16x3_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const u32x4 *>(src[0]), static_cast<const u32x4 *>(src[1]),
                       static_cast<const u32x4 *>(src[2]), static_cast<u32x4 *>(dst[0]), static_cast<u32x4 *>(dst[1]),
                       static_cast<u32x4 *>(dst[2]), n);
    return hip_fail(hipGetLastError(), "three-stream copy kernel launch");
}

pw_status launch_copy(const void *src, void *dst, int64_t nbytes, hipStream_t s) {
    const int64_t n = nbytes / 16;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 16) blocks = 256 * 16;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(copy16_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n);
    return hip_fail(hipGetLastError(), "copy kernel launch");
}

}  // namespace pw
