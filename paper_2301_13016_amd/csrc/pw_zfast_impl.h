// Forward Piacsek-Williams advection on arrays stored z-fastest (column
// major: element (k, j, i) at i*si + j*sj + k): the kernel and its launch
// templates, instantiated per storage type in pw_zfast_{f32,f64,bf16,f16}.hip
// (one translation unit each, so that they compile in parallel), the layout of a model whose
// columns are contiguous (the host model of Sec. 2.1 keeps its fields this
// way).  Same operator and same per-point arithmetic as the x-fastest kernel
// (pw_forward_impl.h), so the two give bit-identical source terms.
//
// The stencil is symmetric under exchanging x with z and u with w, apart from
// where the coefficients sit, so the x-fastest design carries over with the
// axes relabelled:
//   * A wavefront owns 64*PZ consecutive levels (lane l: PZ consecutive
//     levels, one vector load) of RJ consecutive y-rows and marches in x
//     through a chunk of columns i.  One row of one x-plane is one contiguous
//     256*PZ-byte (FP32) access per wavefront instruction.
//   * Neighbours in z are register neighbours inside a lane and DPP wavefront
//     shifts across lanes; the level below lane 0 and above lane 63 come from
//     one extra packed "halo" load per plane and field (lane r: below row r,
//     lane 32+r: above row r), broadcast with readlane.
//   * The vertical coefficients now vary along the lanes and not along the
//     march: each lane loads its PZ levels' tzc1, tzc2, tzd1, tzd2 once.
//     tcx, tcy are kernel arguments.
//   * A ring of four x-planes (i-1, i, i+1 feed column i, i+2 in flight),
//     or five with two planes in flight, rotated by unrolling the march.
//   * Tiles are numbered x-chunk fastest, then level chunk, then y-strip, and
//     each XCD takes one contiguous range: tiles sharing x-planes and halo
//     rows run on the same L2.
//   * Fused epilogue (Epi): out = fma(alpha, F, c), the addends of column ii
//     loaded (non-temporal, read once) ahead of that step's x-plane prefetch,
//     as in the x-fastest kernel.
#pragma once

#include "pw_stencil.h"

namespace pw {
namespace zf {

using namespace dev;

template <typename Tin> struct ZfK {
    using Tc = typename Storage<Tin>::Tc;
    const Tin *u, *v, *w;
    Tc *su, *sv, *sw;
    const Tc *tzc1, *tzc2, *tzd1, *tzd2;
    Tc tcx, tcy;
    int32_t nx, ny, nz, h;
    int64_t in_si, out_si;   // x-plane strides (elements); an x-plane fits in 2 GiB
    int32_t in_sj, out_sj;   // column strides (elements)
    int32_t nkc, nty, nxc, xlen, wpb;
    // fused epilogue (Epi instantiations only): out = c + alpha * F
    const Tc *cu, *cv, *cw;
    Tc alpha;
};

// One x-plane of the tile as loaded: rows 0..RJ+1 are y-rows jj0-1 .. jj0+RJ
// (interior numbering), each the lane's PZ levels in storage precision;
// hu/hv/hw the packed halo levels.
template <typename Tin, int PZ, int RJ> struct ZPlane {
    typename Vec<Tin, PZ>::type u[RJ + 2], v[RJ + 2], w[RJ + 2];
    Tin hu, hv, hw;
};

template <int RJ> struct ZAddr {
    uint32_t roff[RJ + 2];   // byte offset, within an x-plane, of this lane's first level in row r
    uint32_t hoff;           // byte offset of this lane's halo element
    int kcol;                // padded level of the lane's first element
};

template <typename Tin, int PZ, int RJ, bool Full>
__device__ __forceinline__ void load_xplane(ZPlane<Tin, PZ, RJ> &P, const ZfK<Tin> &a, int ip, const ZAddr<RJ> &s,
                                            int last_k) {
    const int64_t pb = static_cast<int64_t>(ip) * a.in_si * static_cast<int64_t>(sizeof(Tin));
    const char *bu = reinterpret_cast<const char *>(a.u) + pb;
    const char *bv = reinterpret_cast<const char *>(a.v) + pb;
    const char *bw = reinterpret_cast<const char *>(a.w) + pb;
#pragma unroll
    for (int r = 0; r < RJ + 2; ++r) {
        load_row<Tin, PZ, Full>(P.u[r], bu, s.roff[r], s.kcol, last_k, a.nz, a.h, PW_HALO_KEEP);
        load_row<Tin, PZ, Full>(P.v[r], bv, s.roff[r], s.kcol, last_k, a.nz, a.h, PW_HALO_KEEP);
        load_row<Tin, PZ, Full>(P.w[r], bw, s.roff[r], s.kcol, last_k, a.nz, a.h, PW_HALO_KEEP);
    }
    P.hu = PW_GLOAD(Tin, bu + s.hoff);
    P.hv = PW_GLOAD(Tin, bv + s.hoff);
    P.hw = PW_GLOAD(Tin, bw + s.hoff);
}

template <typename Tc, int PZ> struct LaneCoeffs {
    Tc z1[PZ], z2[PZ], d1[PZ], d2[PZ];
};

// The epilogue's addends of one output column: RJ rows x PZ levels, levels
// clamped into the column (those past the end are never stored).
template <typename Tc, int PZ, int RJ> struct ZEpi {
    typename Vec<Tc, PZ>::type u[RJ], v[RJ], w[RJ];
};

template <typename Tin, int PZ, int RJ, bool Full>
__device__ __forceinline__ void load_zepi(ZEpi<typename Storage<Tin>::Tc, PZ, RJ> &E, const ZfK<Tin> &a, int ii,
                                          const uint32_t (&ooff)[RJ], int kc) {
    using Tc = typename Storage<Tin>::Tc;
    const int64_t ob = static_cast<int64_t>(ii) * a.out_si * static_cast<int64_t>(sizeof(Tc));
    const char *bu = reinterpret_cast<const char *>(a.cu) + ob;
    const char *bv = reinterpret_cast<const char *>(a.cv) + ob;
    const char *bw = reinterpret_cast<const char *>(a.cw) + ob;
#pragma unroll
    for (int r = 0; r < RJ; ++r) {
        if constexpr (Full || PZ == 1) {
            using VT = typename Vec<Tc, PZ>::type;
            E.u[r] = PW_GLOAD_NT(VT, bu + ooff[r]);
            E.v[r] = PW_GLOAD_NT(VT, bv + ooff[r]);
            E.w[r] = PW_GLOAD_NT(VT, bw + ooff[r]);
        } else {
            // ooff is at level kc = min(kk0, nz-1); levels kc+m clamped to nz-1
#pragma unroll
            for (int m = 0; m < PZ; ++m) {
                const int64_t d = static_cast<int64_t>(min(kc + m, a.nz - 1) - kc) * sizeof(Tc);
                E.u[r][m] = PW_GLOAD_NT(Tc, bu + ooff[r] + d);
                E.v[r][m] = PW_GLOAD_NT(Tc, bv + ooff[r] + d);
                E.w[r][m] = PW_GLOAD_NT(Tc, bw + ooff[r] + d);
            }
        }
    }
}

// Source terms of output column ii (interior numbering) from x-planes ii-1
// (m), ii (c) and ii+1 (p).  Per point the operations and their order are
// those of the x-fastest kernel's level(): there "left/right" is x and the
// planes are z; here "below/above" (KM/KP) is z and the planes are x.
template <typename Tin, int PZ, int RJ, bool Full, bool Epi>
__device__ __forceinline__ void column(const ZPlane<Tin, PZ, RJ> &m, const ZPlane<Tin, PZ, RJ> &c,
                                       const ZPlane<Tin, PZ, RJ> &p, const ZfK<Tin> &a, int ii, bool lane0,
                                       bool lane63, int nvalid, const uint32_t (&ooff)[RJ], const bool (&row_ok)[RJ],
                                       const LaneCoeffs<typename Storage<Tin>::Tc, PZ> &K,
                                       const ZEpi<typename Storage<Tin>::Tc, PZ, RJ> &E) {
    using Tc = typename Storage<Tin>::Tc;
#define G(arr, r, x) Storage<Tin>::widen(comp<Tin, PZ>((arr)[r], (x)))
#define W(hh) Storage<Tin>::widen(hh)
    const Tc tcx = a.tcx, tcy = a.tcy;

    // Levels just below / above this lane's PZ levels, per loaded row, for the
    // arrays whose z-neighbours the stencil reads (unused rows are dropped by
    // the compiler).
    Tc uB[RJ + 2], uA[RJ + 2], vB[RJ + 2], vA[RJ + 2], wB[RJ + 2], wA[RJ + 2], uAm[RJ + 2], wBp[RJ + 2];
#pragma unroll
    for (int r = 0; r < RJ + 2; ++r) {
        uB[r] = left_of(G(c.u, r, PZ - 1), W(c.hu), r, lane0);
        uA[r] = right_of(G(c.u, r, 0), W(c.hu), r, lane63);
        vB[r] = left_of(G(c.v, r, PZ - 1), W(c.hv), r, lane0);
        vA[r] = right_of(G(c.v, r, 0), W(c.hv), r, lane63);
        wB[r] = left_of(G(c.w, r, PZ - 1), W(c.hw), r, lane0);
        wA[r] = right_of(G(c.w, r, 0), W(c.hw), r, lane63);
        uAm[r] = right_of(G(m.u, r, 0), W(m.hu), r, lane63);
        wBp[r] = left_of(G(p.w, r, PZ - 1), W(p.hw), r, lane0);
    }
    // value at (row r, level x-1) / (row r, level x+1) of a plane array
#define KM(arr, B, r, x) ((x) == 0 ? B[r] : G(arr, r, (x) - 1))
#define KP(arr, A, r, x) ((x) == PZ - 1 ? A[r] : G(arr, r, (x) + 1))

    //   fy = v(k,r,i) + v(k,r,i+1)   gy = v(k,r,i) + v(k,r+1,i)   hy = v(k,r,i) + v(k+1,r,i)
    Tc fy[RJ + 1][PZ], gy[RJ + 1][PZ], hy[RJ + 1][PZ];
#pragma unroll
    for (int r = 0; r <= RJ; ++r) {
#pragma unroll
        for (int x = 0; x < PZ; ++x) {
            fy[r][x] = G(c.v, r, x) + G(p.v, r, x);
            gy[r][x] = G(c.v, r, x) + G(c.v, r + 1, x);
            hy[r][x] = G(c.v, r, x) + KP(c.v, vA, r, x);
        }
    }

    const int64_t ob = static_cast<int64_t>(ii) * a.out_si * static_cast<int64_t>(sizeof(Tc));
    char *osu = reinterpret_cast<char *>(a.su) + ob;
    char *osv = reinterpret_cast<char *>(a.sv) + ob;
    char *osw = reinterpret_cast<char *>(a.sw) + ob;

#pragma unroll
    for (int r = 0; r < RJ; ++r) {
        const int q = r + 1;
        Tc rsu[PZ], rsv[PZ], rsw[PZ];
#pragma unroll
        for (int x = 0; x < PZ; ++x) {
            // su
            const Tc uc = G(c.u, q, x);
            const Tc ul = G(m.u, q, x), ur = G(p.u, q, x);
            const Tc ax = fma_(-ur, uc + ur, ul * (uc + ul));
            const Tc ay = fma_(-G(c.u, q + 1, x), fy[q][x], G(c.u, q - 1, x) * fy[r][x]);
            const Tc fzm = KM(c.w, wB, q, x) + KM(p.w, wBp, q, x);
            const Tc fzp = G(c.w, q, x) + G(p.w, q, x);
            Tc su = tcx * ax;
            su = fma_(tcy, ay, su);
            su = fma_(K.z1[x] * KM(c.u, uB, q, x), fzm, su);
            su = fma_(-(K.z2[x] * KP(c.u, uA, q, x)), fzp, su);

            // sv
            const Tc vl = G(m.v, q, x), vr = G(p.v, q, x);
            const Tc gxp = uc + G(c.u, q + 1, x);
            const Tc gxm = ul + G(m.u, q + 1, x);
            const Tc bx = fma_(-vr, gxp, vl * gxm);
            const Tc by = fma_(-G(c.v, q + 1, x), gy[q][x], G(c.v, q - 1, x) * gy[r][x]);
            const Tc gzm = KM(c.w, wB, q, x) + KM(c.w, wB, q + 1, x);
            const Tc gzp = G(c.w, q, x) + G(c.w, q + 1, x);
            Tc sv = tcx * bx;
            sv = fma_(tcy, by, sv);
            sv = fma_(K.z1[x] * KM(c.v, vB, q, x), gzm, sv);
            sv = fma_(-(K.z2[x] * KP(c.v, vA, q, x)), gzp, sv);

            // sw
            const Tc wc = G(c.w, q, x);
            const Tc wl = G(m.w, q, x), wr = G(p.w, q, x);
            const Tc hxp = uc + KP(c.u, uA, q, x);
            const Tc hxm = ul + KP(m.u, uAm, q, x);
            const Tc cx = fma_(-wr, hxp, wl * hxm);
            const Tc cy = fma_(-G(c.w, q + 1, x), hy[q][x], G(c.w, q - 1, x) * hy[r][x]);
            const Tc wkm = KM(c.w, wB, q, x), wkp = KP(c.w, wA, q, x);
            const Tc hzm = wc + wkm;
            const Tc hzp = wc + wkp;
            Tc sw = tcx * cx;
            sw = fma_(tcy, cy, sw);
            sw = fma_(K.d1[x] * wkm, hzm, sw);
            sw = fma_(-(K.d2[x] * wkp), hzp, sw);

            if constexpr (Epi) {   // out = c + alpha * F, one rounding
                su = fma_(a.alpha, su, comp<Tc, PZ>(E.u[r], x));
                sv = fma_(a.alpha, sv, comp<Tc, PZ>(E.v[r], x));
                sw = fma_(a.alpha, sw, comp<Tc, PZ>(E.w[r], x));
            }
            rsu[x] = su;
            rsv[x] = sv;
            rsw[x] = sw;
        }
        if (row_ok[r]) {
            if (Full) {
                (void)nvalid;
                store_vec<Tc, PZ>(osu + ooff[r], rsu);
                store_vec<Tc, PZ>(osv + ooff[r], rsv);
                store_vec<Tc, PZ>(osw + ooff[r], rsw);
            } else {
#pragma unroll
                for (int x = 0; x < PZ; ++x) {
                    if (x < nvalid) {
                        PW_GSTORE(Tc, rsu[x], osu + ooff[r] + x * sizeof(Tc));
                        PW_GSTORE(Tc, rsv[x], osv + ooff[r] + x * sizeof(Tc));
                        PW_GSTORE(Tc, rsw[x], osw + ooff[r] + x * sizeof(Tc));
                    }
                }
            }
        }
    }
#undef KM
#undef KP
#undef G
#undef W
}

// One work item: level chunk tk (64*PZ levels), y-strip ty (RJ rows), marched
// through x-chunk cx.  All 64 lanes must be active.  Full: the level chunk
// lies wholly inside the grid ((tk+1)*64*PZ <= nz), so every lane loads
// whole vectors and owns PZ outputs; otherwise loads are clamped element-wise
// into the column and each lane stores only its levels inside the grid.
template <typename Tin, int PZ, int RJ, bool Full, int Depth, bool Epi>
__device__ __forceinline__ void xmarch(const ZfK<Tin> &a, int tk, int ty, int cx) {
    using Tc = typename Storage<Tin>::Tc;
    const int lane = threadIdx.x & 63;
    const int plev = a.nz + 2 * a.h, prows = a.ny + 2 * a.h;
    const int last_k = plev - 1;
    const int kk0 = tk * 64 * PZ + lane * PZ;   // first interior level of this lane
    const int nvalid = a.nz - kk0;
    const int jj0 = ty * RJ;

    ZAddr<RJ> s;
    s.kcol = min(kk0 + a.h, last_k);
#pragma unroll
    for (int r = 0; r < RJ + 2; ++r) {
        const int prow = min(jj0 - 1 + a.h + r, prows - 1);
        s.roff[r] = static_cast<uint32_t>((prow * a.in_sj + s.kcol) * static_cast<int>(sizeof(Tin)));
    }
    {   // packed halo: lane r -> level below row r, lane 32+r -> level above row r
        const int hr = min(lane & 31, RJ + 1);
        const int hrow = min(jj0 - 1 + a.h + hr, prows - 1);
        const int hk = (lane & 32) ? min(tk * 64 * PZ + 64 * PZ + a.h, last_k) : tk * 64 * PZ + a.h - 1;
        s.hoff = static_cast<uint32_t>((hrow * a.in_sj + hk) * static_cast<int>(sizeof(Tin)));
    }
    uint32_t ooff[RJ];
    bool row_ok[RJ];
    const int kc = min(kk0, a.nz - 1);
#pragma unroll
    for (int r = 0; r < RJ; ++r) {
        row_ok[r] = jj0 + r < a.ny;
        const int jj = min(jj0 + r, a.ny - 1);
        ooff[r] = static_cast<uint32_t>((jj * a.out_sj + kc) * static_cast<int>(sizeof(Tc)));
    }
    LaneCoeffs<Tc, PZ> K;
#pragma unroll
    for (int x = 0; x < PZ; ++x) {
        const int kq = min(kk0 + x, a.nz - 1);
        K.z1[x] = PW_GLOAD(Tc, a.tzc1 + kq);
        K.z2[x] = PW_GLOAD(Tc, a.tzc2 + kq);
        K.d1[x] = PW_GLOAD(Tc, a.tzd1 + kq);
        K.d2[x] = PW_GLOAD(Tc, a.tzd2 + kq);
    }
    const bool lane0 = lane == 0, lane63 = lane == 63;

    const int i0 = cx * a.xlen;
    const int i1 = min(a.nx, i0 + a.xlen);
    const int h = a.h;
    // The prefetch is unconditional and clamped (near the chunk's end it
    // re-reads x-plane i1, a cache hit): a conditional load would merge paths
    // with different loads in flight, and the wait at such a merge drains the
    // prefetch too.
    ZEpi<Tc, PZ, RJ> Ep;   // the epilogue's addends of the current column
    // The addends of column ii are loaded before that step's x-plane prefetch
    // (a scheduling barrier keeps the compiler from moving them after it), so
    // waiting for them never waits for the prefetch.
#define PW_XLOAD(P, ip)                                                      \
    do {                                                                     \
        if constexpr (Epi) {                                                 \
            load_zepi<Tin, PZ, RJ, Full>(Ep, a, ii, ooff, kc);               \
            __builtin_amdgcn_sched_barrier(0);                               \
        }                                                                    \
        load_xplane<Tin, PZ, RJ, Full>(P, a, min((ip), i1) + h, s, last_k); \
    } while (0)
#define PW_XPLOAD(P, ip) load_xplane<Tin, PZ, RJ, Full>(P, a, min((ip), i1) + h, s, last_k)
#define PW_COL(M, C, P) column<Tin, PZ, RJ, Full, Epi>(M, C, P, a, ii, lane0, lane63, nvalid, ooff, row_ok, K, Ep)
    int ii = i0;
    if constexpr (Depth == 1) {
        ZPlane<Tin, PZ, RJ> A, B, C, D;
        load_xplane<Tin, PZ, RJ, Full>(A, a, i0 - 1 + h, s, last_k);
        PW_XPLOAD(B, i0);
        PW_XPLOAD(C, i0 + 1);
        for (;;) {
            PW_XLOAD(D, ii + 2);
            PW_COL(A, B, C);
            if (++ii >= i1) break;
            PW_XLOAD(A, ii + 2);
            PW_COL(B, C, D);
            if (++ii >= i1) break;
            PW_XLOAD(B, ii + 2);
            PW_COL(C, D, A);
            if (++ii >= i1) break;
            PW_XLOAD(C, ii + 2);
            PW_COL(D, A, B);
            if (++ii >= i1) break;
        }
    } else {
        // five-plane ring: x-planes ii+2 and ii+3 in flight
        static_assert(Depth == 2, "prefetch depth 1 or 2");
        ZPlane<Tin, PZ, RJ> A, B, C, D, E;
        load_xplane<Tin, PZ, RJ, Full>(A, a, i0 - 1 + h, s, last_k);
        PW_XPLOAD(B, i0);
        PW_XPLOAD(C, i0 + 1);
        PW_XPLOAD(D, i0 + 2);
        for (;;) {
            PW_XLOAD(E, ii + 3);
            PW_COL(A, B, C);
            if (++ii >= i1) break;
            PW_XLOAD(A, ii + 3);
            PW_COL(B, C, D);
            if (++ii >= i1) break;
            PW_XLOAD(B, ii + 3);
            PW_COL(C, D, E);
            if (++ii >= i1) break;
            PW_XLOAD(C, ii + 3);
            PW_COL(D, E, A);
            if (++ii >= i1) break;
            PW_XLOAD(D, ii + 3);
            PW_COL(E, A, B);
            if (++ii >= i1) break;
        }
    }
#undef PW_XLOAD
#undef PW_XPLOAD
#undef PW_COL
}

template <typename Tin, int PZ, int RJ, int Depth, bool Epi, int MaxT>
__global__ __launch_bounds__(MaxT) void pw_zfast_kernel(ZfK<Tin> a) {
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cx = t % a.nxc;
    const int t2 = t / a.nxc;
    const int tk = t2 % a.nkc;
    const int ty = (t2 / a.nkc) * a.wpb + wave;
    if (ty >= a.nty) return;   // whole wavefront
    if ((tk + 1) * 64 * PZ <= a.nz)
        xmarch<Tin, PZ, RJ, true, Depth, Epi>(a, tk, ty, cx);
    else
        xmarch<Tin, PZ, RJ, false, Depth, Epi>(a, tk, ty, cx);
}

template <typename Tin, int PZ, int RJ, bool Epi>
void launch_k(const ZfK<Tin> &a, const TileCfg &cfg, dim3 grid, dim3 block, hipStream_t s) {
    if (cfg.depth == 2) {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_zfast_kernel<Tin, PZ, RJ, 2, Epi, 256>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_zfast_kernel<Tin, PZ, RJ, 2, Epi, 512>), grid, block, 0, s, a);
    } else {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_zfast_kernel<Tin, PZ, RJ, 1, Epi, 256>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_zfast_kernel<Tin, PZ, RJ, 1, Epi, 512>), grid, block, 0, s, a);
    }
}

template <typename Tin, int PZ, int RJ>
pw_status launch_t(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    using Tc = typename Storage<Tin>::Tc;
    ZfK<Tin> a;
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
    // z-fastest strides travel in the (row, plane) fields of FwdArgs
    a.in_sj = static_cast<int32_t>(g.in_sy);
    a.in_si = g.in_sz;
    a.out_sj = static_cast<int32_t>(g.out_sy);
    a.out_si = g.out_sz;
    a.nkc = static_cast<int32_t>((g.nz + 64 * PZ - 1) / (64 * PZ));
    a.nty = static_cast<int32_t>((g.ny + RJ - 1) / RJ);
    a.xlen = cfg.zlen;
    a.nxc = static_cast<int32_t>((g.nx + cfg.zlen - 1) / cfg.zlen);
    a.wpb = cfg.wpb;
    const int64_t nblk_y = (a.nty + cfg.wpb - 1) / cfg.wpb;
    const int64_t nblocks = static_cast<int64_t>(a.nkc) * nblk_y * a.nxc;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    const dim3 grid(static_cast<unsigned>(nblocks)), block(64 * cfg.wpb);
    a.cu = static_cast<const Tc *>(g.cu);
    a.cv = static_cast<const Tc *>(g.cv);
    a.cw = static_cast<const Tc *>(g.cw);
    a.alpha = static_cast<Tc>(g.alpha);
    if (g.epilogue)
        launch_k<Tin, PZ, RJ, true>(a, cfg, grid, block, s);
    else
        launch_k<Tin, PZ, RJ, false>(a, cfg, grid, block, s);
    return hip_fail(hipGetLastError(), "z-fastest forward kernel launch");
}

template <typename Tin, int PZ>
pw_status launch_pz(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.ry) {
        case 1: return launch_t<Tin, PZ, 1>(g, cfg, s);
        case 2: return launch_t<Tin, PZ, 2>(g, cfg, s);
        case 4:
            if constexpr (PZ <= 2) return launch_t<Tin, PZ, 4>(g, cfg, s);
            [[fallthrough]];
        case 8:
            if constexpr (PZ == 1) return launch_t<Tin, PZ, 8>(g, cfg, s);
            [[fallthrough]];
        default: return fail(PW_ERR_UNSUPPORTED, "rows per strip %d with %d levels per lane not instantiated", cfg.ry, PZ);
    }
}

template <typename Tin>
pw_status launch_dt(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.px) {
        case 1: return launch_pz<Tin, 1>(g, cfg, s);
        case 2: return launch_pz<Tin, 2>(g, cfg, s);
        case 4:
            if constexpr (sizeof(Tin) <= 4) return launch_pz<Tin, 4>(g, cfg, s);
            [[fallthrough]];
        default: return fail(PW_ERR_UNSUPPORTED, "%d levels per lane not instantiated", cfg.px);
    }
}

}  // namespace zf
}  // namespace pw
