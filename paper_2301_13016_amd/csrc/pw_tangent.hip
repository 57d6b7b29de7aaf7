// Tangent-linear operator (Jacobian-vector product) of the PW advection
// operator, gfx950:
//   (tu, tv, tw) = J(u, v, w) (du, dv, dw)
// on the interior.  The operator is a sum of terms s * c * a * (b + d) (a a
// value next to the point, b + d the advecting velocity summed onto a cell
// face), so its derivative in direction (du, dv, dw) is the sum of
//   s * c * (da * (b + d) + a * (db + dd)),
// the product rule applied to every term.  The walk over the grid is the
// forward kernel's strip march (a wavefront owns 64*PX columns x RY rows and
// marches up a z-chunk with a four-plane register ring, x-neighbours by DPP
// and packed halo loads), with two rings: the values and the direction.
// Arithmetic in the storage type (FP32 or FP64), explicit fma, a fixed order
// per point, so results do not depend on the launch shape.
#include "pw_stencil.h"

namespace pw {
namespace {

using namespace dev;

template <typename T> struct TanK {
    FwdK<T> x;                   // values u, v, w; outputs (tu, tv, tw in su, sv, sw); coefficients; shape
    const T *du, *dv, *dw;       // direction, padded like u, v, w
};

// a*(b+d) differentiated: da * s + a * ds with s = b + d, ds = db + dd
template <typename T> __device__ __forceinline__ T tl_term(T a, T da, T s, T ds) { return fma_(da, s, a * ds); }

// Tangent source terms of output level kk from value planes (xm, xc, xp) and
// direction planes (dm, dc, dp) at kk-1, kk, kk+1.
template <typename T, int PX, int RY, bool Full>
__device__ __forceinline__ void level_tl(const Plane<T, PX, RY> &xm, const Plane<T, PX, RY> &xc,
                                         const Plane<T, PX, RY> &xp, const Plane<T, PX, RY> &dm,
                                         const Plane<T, PX, RY> &dc, const Plane<T, PX, RY> &dp, const FwdK<T> &a,
                                         int kk, bool lane0, bool lane63, int nvalid, const uint32_t (&ooff)[RY],
                                         const bool (&row_ok)[RY]) {
#define G(arr, r, x) comp<T, PX>((arr)[r], (x))
    const T z1 = uniform_load(a.tzc1, kk), z2 = uniform_load(a.tzc2, kk);
    const T d1 = uniform_load(a.tzd1, kk), d2 = uniform_load(a.tzd2, kk);
    const T tcx = a.tcx, tcy = a.tcy;

    // Columns just outside the lane's PX columns (values X.., direction D..).
    T XuL[RY + 2], XuR[RY + 2], XvL[RY + 2], XvR[RY + 2], XwL[RY + 2], XwR[RY + 2], XwRm[RY + 2], XuLp[RY + 2];
    T DuL[RY + 2], DuR[RY + 2], DvL[RY + 2], DvR[RY + 2], DwL[RY + 2], DwR[RY + 2], DwRm[RY + 2], DuLp[RY + 2];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        XuL[r] = left_of(G(xc.u, r, PX - 1), xc.hu, r, lane0);
        XuR[r] = right_of(G(xc.u, r, 0), xc.hu, r, lane63);
        XvL[r] = left_of(G(xc.v, r, PX - 1), xc.hv, r, lane0);
        XvR[r] = right_of(G(xc.v, r, 0), xc.hv, r, lane63);
        XwL[r] = left_of(G(xc.w, r, PX - 1), xc.hw, r, lane0);
        XwR[r] = right_of(G(xc.w, r, 0), xc.hw, r, lane63);
        XwRm[r] = right_of(G(xm.w, r, 0), xm.hw, r, lane63);
        XuLp[r] = left_of(G(xp.u, r, PX - 1), xp.hu, r, lane0);
        DuL[r] = left_of(G(dc.u, r, PX - 1), dc.hu, r, lane0);
        DuR[r] = right_of(G(dc.u, r, 0), dc.hu, r, lane63);
        DvL[r] = left_of(G(dc.v, r, PX - 1), dc.hv, r, lane0);
        DvR[r] = right_of(G(dc.v, r, 0), dc.hv, r, lane63);
        DwL[r] = left_of(G(dc.w, r, PX - 1), dc.hw, r, lane0);
        DwR[r] = right_of(G(dc.w, r, 0), dc.hw, r, lane63);
        DwRm[r] = right_of(G(dm.w, r, 0), dm.hw, r, lane63);
        DuLp[r] = left_of(G(dp.u, r, PX - 1), dp.hu, r, lane0);
    }
#define XM(arr, L, r, x) ((x) == 0 ? L[r] : G(arr, r, (x) - 1))
#define XP(arr, R, r, x) ((x) == PX - 1 ? R[r] : G(arr, r, (x) + 1))

    // Face sums shared by consecutive rows (index r = loaded row), values and direction:
    //   fy = v(k,r,i) + v(k,r,i+1)   gy = v(k,r,i) + v(k,r+1,i)   hy = v(k,r,i) + v(k+1,r,i)
    T fy[RY + 1][PX], gy[RY + 1][PX], hy[RY + 1][PX];
    T dfy[RY + 1][PX], dgy[RY + 1][PX], dhy[RY + 1][PX];
#pragma unroll
    for (int r = 0; r <= RY; ++r) {
#pragma unroll
        for (int x = 0; x < PX; ++x) {
            fy[r][x] = G(xc.v, r, x) + XP(xc.v, XvR, r, x);
            gy[r][x] = G(xc.v, r, x) + G(xc.v, r + 1, x);
            hy[r][x] = G(xc.v, r, x) + G(xp.v, r, x);
            dfy[r][x] = G(dc.v, r, x) + XP(dc.v, DvR, r, x);
            dgy[r][x] = G(dc.v, r, x) + G(dc.v, r + 1, x);
            dhy[r][x] = G(dc.v, r, x) + G(dp.v, r, x);
        }
    }

    const int64_t ob = static_cast<int64_t>(kk) * a.out_sz * static_cast<int64_t>(sizeof(T));
    char *otu = reinterpret_cast<char *>(a.su) + ob;
    char *otv = reinterpret_cast<char *>(a.sv) + ob;
    char *otw = reinterpret_cast<char *>(a.sw) + ob;

#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int q = r + 1;   // this output row within the loaded rows
        T rtu[PX], rtv[PX], rtw[PX];
#pragma unroll
        for (int x = 0; x < PX; ++x) {
            // tu: x faces (u+u), y faces (v+v at i, i+1), z faces (w+w at i, i+1)
            const T uc = G(xc.u, q, x), duc = G(dc.u, q, x);
            const T ul = XM(xc.u, XuL, q, x), dul = XM(dc.u, DuL, q, x);
            const T ur = XP(xc.u, XuR, q, x), dur = XP(dc.u, DuR, q, x);
            const T ax = tl_term(ul, dul, uc + ul, duc + dul) - tl_term(ur, dur, uc + ur, duc + dur);
            const T ay = tl_term(G(xc.u, q - 1, x), G(dc.u, q - 1, x), fy[r][x], dfy[r][x]) -
                         tl_term(G(xc.u, q + 1, x), G(dc.u, q + 1, x), fy[q][x], dfy[q][x]);
            const T fzm = G(xm.w, q, x) + XP(xm.w, XwRm, q, x), dfzm = G(dm.w, q, x) + XP(dm.w, DwRm, q, x);
            const T fzp = G(xc.w, q, x) + XP(xc.w, XwR, q, x), dfzp = G(dc.w, q, x) + XP(dc.w, DwR, q, x);
            T tu = tcx * ax;
            tu = fma_(tcy, ay, tu);
            tu = fma_(z1, tl_term(G(xm.u, q, x), G(dm.u, q, x), fzm, dfzm), tu);
            tu = fma_(-z2, tl_term(G(xp.u, q, x), G(dp.u, q, x), fzp, dfzp), tu);

            // tv: x faces (u+u at j, j+1), y faces (v+v), z faces (w+w at j, j+1)
            const T vl = XM(xc.v, XvL, q, x), dvl = XM(dc.v, DvL, q, x);
            const T vr = XP(xc.v, XvR, q, x), dvr = XP(dc.v, DvR, q, x);
            const T gxp = uc + G(xc.u, q + 1, x), dgxp = duc + G(dc.u, q + 1, x);
            const T gxm = ul + XM(xc.u, XuL, q + 1, x), dgxm = dul + XM(dc.u, DuL, q + 1, x);
            const T bx = tl_term(vl, dvl, gxm, dgxm) - tl_term(vr, dvr, gxp, dgxp);
            const T by = tl_term(G(xc.v, q - 1, x), G(dc.v, q - 1, x), gy[r][x], dgy[r][x]) -
                         tl_term(G(xc.v, q + 1, x), G(dc.v, q + 1, x), gy[q][x], dgy[q][x]);
            const T gzm = G(xm.w, q, x) + G(xm.w, q + 1, x), dgzm = G(dm.w, q, x) + G(dm.w, q + 1, x);
            const T gzp = G(xc.w, q, x) + G(xc.w, q + 1, x), dgzp = G(dc.w, q, x) + G(dc.w, q + 1, x);
            T tv = tcx * bx;
            tv = fma_(tcy, by, tv);
            tv = fma_(z1, tl_term(G(xm.v, q, x), G(dm.v, q, x), gzm, dgzm), tv);
            tv = fma_(-z2, tl_term(G(xp.v, q, x), G(dp.v, q, x), gzp, dgzp), tv);

            // tw: x faces (u+u at k, k+1), y faces (v+v at k, k+1), z faces (w+w)
            const T wc = G(xc.w, q, x), dwc = G(dc.w, q, x);
            const T wl = XM(xc.w, XwL, q, x), dwl = XM(dc.w, DwL, q, x);
            const T wr = XP(xc.w, XwR, q, x), dwr = XP(dc.w, DwR, q, x);
            const T hxp = uc + G(xp.u, q, x), dhxp = duc + G(dp.u, q, x);
            const T hxm = ul + XM(xp.u, XuLp, q, x), dhxm = dul + XM(dp.u, DuLp, q, x);
            const T cx = tl_term(wl, dwl, hxm, dhxm) - tl_term(wr, dwr, hxp, dhxp);
            const T cy = tl_term(G(xc.w, q - 1, x), G(dc.w, q - 1, x), hy[r][x], dhy[r][x]) -
                         tl_term(G(xc.w, q + 1, x), G(dc.w, q + 1, x), hy[q][x], dhy[q][x]);
            const T hzm = wc + G(xm.w, q, x), dhzm = dwc + G(dm.w, q, x);
            const T hzp = wc + G(xp.w, q, x), dhzp = dwc + G(dp.w, q, x);
            T tw = tcx * cx;
            tw = fma_(tcy, cy, tw);
            tw = fma_(d1, tl_term(G(xm.w, q, x), G(dm.w, q, x), hzm, dhzm), tw);
            tw = fma_(-d2, tl_term(G(xp.w, q, x), G(dp.w, q, x), hzp, dhzp), tw);

            rtu[x] = tu;
            rtv[x] = tv;
            rtw[x] = tw;
        }
        if (row_ok[r]) {
            if (Full) {
                (void)nvalid;
                store_vec<T, PX>(otu + ooff[r], rtu);
                store_vec<T, PX>(otv + ooff[r], rtv);
                store_vec<T, PX>(otw + ooff[r], rtw);
            } else {
#pragma unroll
                for (int x = 0; x < PX; ++x) {
                    if (x < nvalid) {
                        reinterpret_cast<T *>(otu + ooff[r])[x] = rtu[x];
                        reinterpret_cast<T *>(otv + ooff[r])[x] = rtv[x];
                        reinterpret_cast<T *>(otw + ooff[r])[x] = rtw[x];
                    }
                }
            }
        }
    }
#undef G
#undef XM
#undef XP
}

// One work item: strip (tx, ty) of the tangent marched up z-chunk cz (the
// forward kernel's march, loading the value and direction planes together;
// see strip_march_t for the ring and the unconditional prefetch).  Depth:
// planes in flight ahead of the three a level reads (1 or 2).
template <typename T, int PX, int RY, int Depth, bool Full>
__device__ __forceinline__ void tl_march(const FwdK<T> &a, const FwdK<T> &d, int tx, int ty, int cz) {
    const int lane = threadIdx.x & 63;
    const int pcols = a.nx + 2 * a.h, prows = a.ny + 2 * a.h;
    const int last_col = pcols - 1;
    const int ii0 = tx * 64 * PX + lane * PX;
    const int nvalid = a.nx - ii0;
    const int jj0 = ty * RY;

    StripAddr<RY> s;
    s.col = min(ii0 + a.h, last_col);
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int prow = min(jj0 - 1 + a.h + r, prows - 1);
        s.roff[r] = static_cast<uint32_t>((prow * a.in_sy + s.col) * static_cast<int>(sizeof(T)));
    }
    {
        const int hr = min(lane & 31, RY + 1);
        const int hrow = min(jj0 - 1 + a.h + hr, prows - 1);
        const int hcol = (lane & 32) ? min(tx * 64 * PX + 64 * PX + a.h, last_col) : tx * 64 * PX + a.h - 1;
        s.hoff = static_cast<uint32_t>((hrow * a.in_sy + hcol) * static_cast<int>(sizeof(T)));
    }
    uint32_t ooff[RY];
    bool row_ok[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row_ok[r] = jj0 + r < a.ny;
        const int jj = min(jj0 + r, a.ny - 1);
        const int ic = min(ii0, a.nx - 1);
        ooff[r] = static_cast<uint32_t>((jj * a.out_sy + ic) * static_cast<int>(sizeof(T)));
    }
    const bool lane0 = lane == 0, lane63 = lane == 63;
    const int k0 = cz * a.zlen;
    const int k1 = min(a.nz, k0 + a.zlen);
    const int h = a.h;

#define PW_LOAD(Xp, Dp, kp)                                          \
    do {                                                             \
        load_plane<T, PX, RY, Full>(Xp, a, (kp), s, last_col);       \
        load_plane<T, PX, RY, Full>(Dp, d, (kp), s, last_col);       \
    } while (0)
#define PW_LEVEL(M, C, P) \
    level_tl<T, PX, RY, Full>(X##M, X##C, X##P, D##M, D##C, D##P, a, kk, lane0, lane63, nvalid, ooff, row_ok)
    int kk = k0;
    if constexpr (Depth == 1) {
        // four-plane rings: planes kk-1, kk, kk+1 feed level kk, kk+2 in flight
        Plane<T, PX, RY> XA, XB, XC, XD, DA, DB, DC, DD;
        PW_LOAD(XA, DA, k0 - 1 + h);
        PW_LOAD(XB, DB, k0 + h);
        PW_LOAD(XC, DC, k0 + 1 + h);
        for (;;) {
            PW_LOAD(XD, DD, min(kk + 2, k1) + h);
            PW_LEVEL(A, B, C);
            if (++kk >= k1) break;
            PW_LOAD(XA, DA, min(kk + 2, k1) + h);
            PW_LEVEL(B, C, D);
            if (++kk >= k1) break;
            PW_LOAD(XB, DB, min(kk + 2, k1) + h);
            PW_LEVEL(C, D, A);
            if (++kk >= k1) break;
            PW_LOAD(XC, DC, min(kk + 2, k1) + h);
            PW_LEVEL(D, A, B);
            if (++kk >= k1) break;
        }
    } else {
        // five-plane rings: planes kk+2 and kk+3 in flight
        static_assert(Depth == 2, "prefetch depth 1 or 2");
        Plane<T, PX, RY> XA, XB, XC, XD, XE, DA, DB, DC, DD, DE;
        PW_LOAD(XA, DA, k0 - 1 + h);
        PW_LOAD(XB, DB, k0 + h);
        PW_LOAD(XC, DC, k0 + 1 + h);
        PW_LOAD(XD, DD, min(k0 + 2, k1) + h);
        for (;;) {
            PW_LOAD(XE, DE, min(kk + 3, k1) + h);
            PW_LEVEL(A, B, C);
            if (++kk >= k1) break;
            PW_LOAD(XA, DA, min(kk + 3, k1) + h);
            PW_LEVEL(B, C, D);
            if (++kk >= k1) break;
            PW_LOAD(XB, DB, min(kk + 3, k1) + h);
            PW_LEVEL(C, D, E);
            if (++kk >= k1) break;
            PW_LOAD(XC, DC, min(kk + 3, k1) + h);
            PW_LEVEL(D, E, A);
            if (++kk >= k1) break;
            PW_LOAD(XD, DD, min(kk + 3, k1) + h);
            PW_LEVEL(E, A, B);
            if (++kk >= k1) break;
        }
    }
#undef PW_LOAD
#undef PW_LEVEL
}

// MaxT: workgroup size bound (built for 256 and 512 threads, as the forward).
template <typename T, int PX, int RY, int Depth, int MaxT>
__global__ __launch_bounds__(MaxT) void pw_tangent_kernel(TanK<T> k) {
    const FwdK<T> &a = k.x;
    FwdK<T> d = k.x;
    d.u = k.du;
    d.v = k.dv;
    d.w = k.dw;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cz = t % a.nzc;
    const int t2 = t / a.nzc;
    const int tx = t2 % a.ntx;
    const int ty = (t2 / a.ntx) * a.wpb + wave;
    if (ty >= a.nty) return;   // whole wavefront
    if constexpr (PX == 1) {
        tl_march<T, PX, RY, Depth, false>(a, d, tx, ty, cz);
    } else if ((tx + 1) * 64 * PX <= a.nx) {
        tl_march<T, PX, RY, Depth, true>(a, d, tx, ty, cz);
    } else {
        tl_march<T, PX, RY, Depth, false>(a, d, tx, ty, cz);
    }
}

template <typename T, int PX, int RY>
pw_status launch_tl_t(const TanArgs &g, const TileCfg &cfg, hipStream_t s) {
    TanK<T> k;
    FwdK<T> &a = k.x;
    a.u = static_cast<const T *>(g.f.u);
    a.v = static_cast<const T *>(g.f.v);
    a.w = static_cast<const T *>(g.f.w);
    a.su = static_cast<T *>(g.f.su);
    a.sv = static_cast<T *>(g.f.sv);
    a.sw = static_cast<T *>(g.f.sw);
    a.tzc1 = static_cast<const T *>(g.f.tzc1);
    a.tzc2 = static_cast<const T *>(g.f.tzc2);
    a.tzd1 = static_cast<const T *>(g.f.tzd1);
    a.tzd2 = static_cast<const T *>(g.f.tzd2);
    a.tcx = static_cast<T>(g.f.tcx);
    a.tcy = static_cast<T>(g.f.tcy);
    a.nx = static_cast<int32_t>(g.f.nx);
    a.ny = static_cast<int32_t>(g.f.ny);
    a.nz = static_cast<int32_t>(g.f.nz);
    a.h = g.f.h;
    a.in_sz = g.f.in_sz;
    a.out_sz = g.f.out_sz;
    a.in_sy = static_cast<int32_t>(g.f.in_sy);
    a.out_sy = static_cast<int32_t>(g.f.out_sy);
    a.ntx = static_cast<int32_t>((g.f.nx + 64 * PX - 1) / (64 * PX));
    a.nty = static_cast<int32_t>((g.f.ny + RY - 1) / RY);
    a.zlen = cfg.zlen;
    a.nzc = static_cast<int32_t>((g.f.nz + cfg.zlen - 1) / cfg.zlen);
    a.wpb = cfg.wpb;
    k.du = static_cast<const T *>(g.du);
    k.dv = static_cast<const T *>(g.dv);
    k.dw = static_cast<const T *>(g.dw);
    const int64_t nblk_y = (a.nty + cfg.wpb - 1) / cfg.wpb;
    const int64_t nblocks = static_cast<int64_t>(a.ntx) * nblk_y * a.nzc;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    const dim3 grid(static_cast<unsigned>(nblocks)), block(64 * cfg.wpb);
    if (cfg.depth == 2) {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_tangent_kernel<T, PX, RY, 2, 256>), grid, block, 0, s, k);
        else
            hipLaunchKernelGGL((pw_tangent_kernel<T, PX, RY, 2, 512>), grid, block, 0, s, k);
    } else {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_tangent_kernel<T, PX, RY, 1, 256>), grid, block, 0, s, k);
        else
            hipLaunchKernelGGL((pw_tangent_kernel<T, PX, RY, 1, 512>), grid, block, 0, s, k);
    }
    return hip_fail(hipGetLastError(), "tangent kernel launch");
}

template <typename T, int PX>
pw_status launch_tl_px(const TanArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.ry) {
        case 1: return launch_tl_t<T, PX, 1>(g, cfg, s);
        case 2: return launch_tl_t<T, PX, 2>(g, cfg, s);
        default: return fail(PW_ERR_UNSUPPORTED, "tangent rows per strip %d not instantiated", cfg.ry);
    }
}

template <typename T>
pw_status launch_tl_dt(const TanArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.px) {
        case 1: return launch_tl_px<T, 1>(g, cfg, s);
        case 2:
            if constexpr (sizeof(T) == 4) return launch_tl_px<T, 2>(g, cfg, s);
            [[fallthrough]];
        default: return fail(PW_ERR_UNSUPPORTED, "tangent columns per lane %d not instantiated", cfg.px);
    }
}

}  // namespace

bool tangent_tile_supported(const TileCfg &c, pw_dtype dt) {
    if (c.zlen < 1 || c.wpb < 1 || c.wpb > 8 || (c.depth != 1 && c.depth != 2) || c.share != 0) return false;
    if (c.ry != 1 && c.ry != 2) return false;
    if (dt == PW_F64) return c.px == 1;
    return c.px == 1 || c.px == 2;
}

TileCfg default_tangent_tile(const TanArgs &a, pw_dtype dt) {
    // two-row strips of 64 (FP32: 128) columns, about 2048 wavefronts in flight
    TileCfg c;
    c.px = (dt == PW_F64) ? 1 : 2;
    c.ry = 2;
    c.wpb = 1;
    const int64_t strips = ((a.f.nx + 64 * c.px - 1) / (64 * c.px)) * ((a.f.ny + c.ry - 1) / c.ry);
    int64_t chunks = (2048 + strips - 1) / strips;
    if (chunks < 1) chunks = 1;
    int64_t zl = (a.f.nz + chunks - 1) / chunks;
    if (zl < 8) zl = 8;
    if (zl > a.f.nz) zl = a.f.nz;
    c.zlen = static_cast<int>(zl);
    return c;
}

pw_status launch_tangent(const TanArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s) {
    if (!tangent_tile_supported(cfg, dt)) return fail(PW_ERR_INVALID_ARG, "unsupported tangent tile configuration");
    switch (dt) {
        case PW_F32: return launch_tl_dt<float>(a, cfg, s);
        case PW_F64: return launch_tl_dt<double>(a, cfg, s);
        default: return fail(PW_ERR_UNSUPPORTED, "tangent dtype %d", static_cast<int>(dt));
    }
}

}  // namespace pw
