// Forward Piacsek-Williams advection kernel for gfx950 (CDNA4): the kernel
// and its launch templates, instantiated per storage type in
// pw_forward_{f32,f64,bf16,f16}.hip (one translation unit each, so that the
// instantiations compile in parallel).
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
#pragma once

#include "pw_stencil.h"

namespace pw {
namespace fwd {

using namespace dev;

// Depth: planes in flight ahead of the level being computed (1 or 2).
// Epi: fused epilogue, out = c + alpha * F (accumulation into the outputs
// when c is the output itself, or a time update c + dt * F).
// Bc: boundary rules applied by addressing (pw_advect_bc): 1 remaps reads
// (periodic, nearest interior), 2 also applies the value rules (zero,
// negation); the plain instantiations (0) carry no mapping code.
// MaxT: the workgroup size bound the kernel is compiled for.  Every shape is
// built twice: for up to 256 threads (four wavefronts, one per SIMD, so a
// wavefront may use the whole 512-entry register file: the large strips keep
// their planes in registers instead of spilling) and for up to 512.
template <typename Tin, int PX, int RY, int Depth, bool Epi, int Bc, int MaxT>
__global__ __launch_bounds__(MaxT) void pw_forward_kernel(FwdK<Tin> a) {
    // wavefront index as a scalar, so that per-strip conditions stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cz = t % a.nzc;
    const int t2 = t / a.nzc;
    const int tx = t2 % a.ntx;
    const int ty = (t2 / a.ntx) * a.wpb + wave;
    if (ty >= a.nty) return;   // whole wavefront
    strip_march<Tin, PX, RY, Depth, Epi, Bc>(a, tx, ty, cz);
}

// W wavefronts per workgroup sharing their edge rows through LDS (see
// strip_march_lds): the workgroup covers W consecutive strips in y.  Every
// wavefront runs, also one whose strip lies past the grid, so that all reach
// the same barriers.
template <typename Tin, int PX, int RY, int Depth, bool Epi, int Bc, int W, bool NtOwn = false>
__global__ __launch_bounds__(64 * W) void pw_forward_lds_kernel(FwdK<Tin> a) {
    __shared__ EdgeLds<Tin, PX, W> L;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cz = t % a.nzc;
    const int t2 = t / a.nzc;
    const int tx = t2 % a.ntx;
    const int ty = (t2 / a.ntx) * W + wave;
    strip_march_lds<Tin, PX, RY, Depth, Epi, Bc, W, NtOwn>(a, L, tx, ty, cz, wave);
}

template <typename Tin, int PX, int RY, bool Epi, int Bc>
void launch_fwd_b(const FwdK<Tin> &a, const TileCfg &cfg, dim3 grid, dim3 block, hipStream_t s) {
    if constexpr (Bc != 0) {   // boundary rules: built for up to four wavefronts per workgroup only
        if (cfg.depth == 2)
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 2, Epi, Bc, 256>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 1, Epi, Bc, 256>), grid, block, 0, s, a);
    } else if (cfg.depth == 2) {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 2, Epi, Bc, 256>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 2, Epi, Bc, 512>), grid, block, 0, s, a);
    } else {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 1, Epi, Bc, 256>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY, 1, Epi, Bc, 512>), grid, block, 0, s, a);
    }
}

template <typename Tin, int PX, int RY, bool Epi>
void launch_fwd_k(const FwdK<Tin> &a, const TileCfg &cfg, dim3 grid, dim3 block, hipStream_t s) {
    if (a.bcv != 0)
        launch_fwd_b<Tin, PX, RY, Epi, 2>(a, cfg, grid, block, s);
    else if (a.bcx != PW_HALO_KEEP || a.bcy != PW_HALO_KEEP || a.bcz != PW_HALO_KEEP)
        launch_fwd_b<Tin, PX, RY, Epi, 1>(a, cfg, grid, block, s);
    else
        launch_fwd_b<Tin, PX, RY, Epi, 0>(a, cfg, grid, block, s);
}

template <typename Tin, int PX, int RY>
FwdK<Tin> make_fwdk(const FwdArgs &g, const TileCfg &cfg) {
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
    a.cu = static_cast<const Tc *>(g.cu);
    a.cv = static_cast<const Tc *>(g.cv);
    a.cw = static_cast<const Tc *>(g.cw);
    a.alpha = static_cast<Tc>(g.alpha);
    a.bcx = g.bcx;
    a.bcy = g.bcy;
    a.bcz = g.bcz;
    a.bcv = g.bcv;
    return a;
}

template <typename Tin, int PX, int RY>
pw_status launch_fwd_t(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    const FwdK<Tin> a = make_fwdk<Tin, PX, RY>(g, cfg);
    const int64_t nblk_y = (a.nty + cfg.wpb - 1) / cfg.wpb;
    const int64_t nblocks = static_cast<int64_t>(a.ntx) * nblk_y * a.nzc;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    const dim3 grid(static_cast<unsigned>(nblocks)), block(64 * cfg.wpb);
    if (g.epilogue)
        launch_fwd_k<Tin, PX, RY, true>(a, cfg, grid, block, s);
    else
        launch_fwd_k<Tin, PX, RY, false>(a, cfg, grid, block, s);
    return hip_fail(hipGetLastError(), "forward kernel launch");
}

template <typename Tin, int PX>
pw_status launch_fwd_px(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.ry) {
        case 1: return launch_fwd_t<Tin, PX, 1>(g, cfg, s);
        case 2: return launch_fwd_t<Tin, PX, 2>(g, cfg, s);
        case 4:
            if constexpr (PX <= 2 || (sizeof(Tin) <= 4 && PX == 4))
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

// Shared-row tiles (cfg.share 1 or 2; see strip_march_lds).  Launched with
// exactly W wavefronts per workgroup.
template <typename Tin, int PX, int RY, int W, bool NtOwn, int Bc>
void launch_lds_b(const FwdK<Tin> &a, bool epi, dim3 grid, dim3 block, hipStream_t s) {
    if (epi)
        hipLaunchKernelGGL((pw_forward_lds_kernel<Tin, PX, RY, 1, true, Bc, W, NtOwn>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((pw_forward_lds_kernel<Tin, PX, RY, 1, false, Bc, W, NtOwn>), grid, block, 0, s, a);
}

template <typename Tin, int PX, int RY, int W, bool NtOwn>
pw_status launch_lds_w(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    const FwdK<Tin> a = make_fwdk<Tin, PX, RY>(g, cfg);
    const int64_t nblk_y = (a.nty + W - 1) / W;
    const int64_t nblocks = static_cast<int64_t>(a.ntx) * nblk_y * a.nzc;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    const dim3 grid(static_cast<unsigned>(nblocks)), block(64 * W);
    if constexpr (W == 4 && NtOwn) {   // the only instantiation that carries boundary rules
        if (a.bcv != 0)
            launch_lds_b<Tin, PX, RY, W, true, 2>(a, g.epilogue, grid, block, s);
        else if (a.bcx != PW_HALO_KEEP || a.bcy != PW_HALO_KEEP || a.bcz != PW_HALO_KEEP)
            launch_lds_b<Tin, PX, RY, W, true, 1>(a, g.epilogue, grid, block, s);
        else
            launch_lds_b<Tin, PX, RY, W, true, 0>(a, g.epilogue, grid, block, s);
    } else {
        launch_lds_b<Tin, PX, RY, W, NtOwn, 0>(a, g.epilogue, grid, block, s);
    }
    return hip_fail(hipGetLastError(), "forward kernel launch");
}

template <typename Tin, int PX, int RY>
pw_status launch_lds_t(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    // boundary rules by addressing: four wavefronts, non-temporal own rows
    // (the grouping of strips and the cache hint change no result)
    if (g.bcx != PW_HALO_KEEP || g.bcy != PW_HALO_KEEP || g.bcz != PW_HALO_KEEP || g.bcv != 0)
        return launch_lds_w<Tin, PX, RY, 4, true>(g, cfg, s);
    const bool nt = cfg.share == 2;
    if (cfg.wpb == 2) return nt ? launch_lds_w<Tin, PX, RY, 2, true>(g, cfg, s) : launch_lds_w<Tin, PX, RY, 2, false>(g, cfg, s);
    if (cfg.wpb == 4) return nt ? launch_lds_w<Tin, PX, RY, 4, true>(g, cfg, s) : launch_lds_w<Tin, PX, RY, 4, false>(g, cfg, s);
    return fail(PW_ERR_UNSUPPORTED, "shared rows with %d wavefronts per workgroup not instantiated", cfg.wpb);
}

}  // namespace fwd
}  // namespace pw
