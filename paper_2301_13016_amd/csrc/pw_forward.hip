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
#include "pw_internal.h"

namespace pw {
namespace {

// ----------------------------------------------------------------- storage
template <typename Tin> struct Storage;
template <> struct Storage<float> {
    using Tc = float;
    static __device__ __forceinline__ float widen(float x) { return x; }
};
template <> struct Storage<double> {
    using Tc = double;
    static __device__ __forceinline__ double widen(double x) { return x; }
};
template <> struct Storage<uint16_t> {   // BF16: the upper half of an FP32 pattern
    using Tc = float;
    static __device__ __forceinline__ float widen(uint16_t x) {
        return __uint_as_float(static_cast<uint32_t>(x) << 16);
    }
};
template <> struct Storage<_Float16> {
    using Tc = float;
    static __device__ __forceinline__ float widen(_Float16 x) { return static_cast<float>(x); }
};

// N consecutive elements, aligned only to the element: the type of one
// lane's vector load or store.
template <typename T, int N> struct Vec;
template <typename T> struct Vec<T, 1> { using type = T; };
template <> struct Vec<float, 2> { typedef float type __attribute__((ext_vector_type(2), aligned(4))); };
template <> struct Vec<float, 4> { typedef float type __attribute__((ext_vector_type(4), aligned(4))); };
template <> struct Vec<double, 2> { typedef double type __attribute__((ext_vector_type(2), aligned(8))); };
template <> struct Vec<uint16_t, 2> { typedef uint16_t type __attribute__((ext_vector_type(2), aligned(2))); };
template <> struct Vec<uint16_t, 4> { typedef uint16_t type __attribute__((ext_vector_type(4), aligned(2))); };
template <> struct Vec<_Float16, 2> { typedef _Float16 type __attribute__((ext_vector_type(2), aligned(2))); };
template <> struct Vec<_Float16, 4> { typedef _Float16 type __attribute__((ext_vector_type(4), aligned(2))); };

template <typename T, int N>
__device__ __forceinline__ T comp(const typename Vec<T, N>::type &v, int m) {
    if constexpr (N == 1) {
        (void)m;
        return v;
    } else {
        return v[m];
    }
}

// ------------------------------------------------------- cross-lane moves
// DPP controls (GFX9 family): wave_shr:1 moves lane l-1 into lane l,
// wave_shl:1 moves lane l+1 into lane l (bound_ctrl: the lane with no source
// reads 0 and is patched from the halo).
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
// Column left of this lane's first column: the previous lane's last value,
// or for lane 0 the strip's left halo (held by lane `row` of `halo`).
template <typename T> __device__ __forceinline__ T left_of(T last, T halo, int row, bool lane0) {
    const T s = wave_shift<kWaveShr1>(last);
    const T h = lane_value(halo, row);
    return lane0 ? h : s;
}
// Column right of this lane's last column (lane 63: right halo, lane 32+row).
template <typename T> __device__ __forceinline__ T right_of(T first, T halo, int row, bool lane63) {
    const T s = wave_shift<kWaveShl1>(first);
    const T h = lane_value(halo, 32 + row);
    return lane63 ? h : s;
}

template <typename T> __device__ __forceinline__ T fma_(T a, T b, T c);
template <> __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// --------------------------------------------------------- kernel operands
template <typename Tin> struct FwdK {
    using Tc = typename Storage<Tin>::Tc;
    const Tin *u, *v, *w;
    Tc *su, *sv, *sw;
    const Tc *tzc1, *tzc2, *tzd1, *tzd2;
    Tc tcx, tcy;
    int32_t nx, ny, nz, h;
    int64_t in_sz, out_sz;     // plane strides (elements)
    int32_t in_sy, out_sy;     // row strides (elements); a plane fits in 2 GiB
    int32_t ntx, nty, nzc, zlen, wpb;
};

// One z-plane of the strip, widened: rows 0..RY+1 are the strip's rows
// jj0-1 .. jj0+RY (interior numbering), PX columns of this lane each; hu/hv/hw
// are the packed halo columns (see left_of / right_of).
template <typename Tc, int PX, int RY> struct Plane {
    Tc u[RY + 2][PX], v[RY + 2][PX], w[RY + 2][PX];
    Tc hu, hv, hw;
};

// Per-lane addressing of the strip, fixed for the whole march.
template <int RY> struct StripAddr {
    uint32_t roff[RY + 2];   // byte offset of this lane's first column in row r
    uint32_t hoff;           // byte offset of this lane's halo element
    int col;                 // padded column of the lane's first element
};

// PX consecutive elements of one row starting at padded column `col`; lanes
// whose vector would run past the row's last column read element-wise with
// the columns clamped (every column a stored output reads is in range, so
// clamping only ever affects values that are not used).
template <typename Tin, int PX>
__device__ __forceinline__ void load_row(typename Storage<Tin>::Tc (&dst)[PX], const char *plane, uint32_t off,
                                         int col, int last_col) {
    if (col + PX - 1 <= last_col) {
        const auto x = *reinterpret_cast<const typename Vec<Tin, PX>::type *>(plane + off);
#pragma unroll
        for (int m = 0; m < PX; ++m) dst[m] = Storage<Tin>::widen(comp<Tin, PX>(x, m));
    } else {
        const char *row = plane + off - static_cast<int64_t>(col) * static_cast<int64_t>(sizeof(Tin));
#pragma unroll
        for (int m = 0; m < PX; ++m)
            dst[m] = Storage<Tin>::widen(
                *reinterpret_cast<const Tin *>(row + static_cast<int64_t>(min(col + m, last_col)) * sizeof(Tin)));
    }
}

template <typename Tin, int PX, int RY>
__device__ __forceinline__ void load_plane(Plane<typename Storage<Tin>::Tc, PX, RY> &P, const FwdK<Tin> &a,
                                           int kp, const StripAddr<RY> &s, int last_col) {
    const int64_t pb = static_cast<int64_t>(kp) * a.in_sz * static_cast<int64_t>(sizeof(Tin));
    const char *bu = reinterpret_cast<const char *>(a.u) + pb;
    const char *bv = reinterpret_cast<const char *>(a.v) + pb;
    const char *bw = reinterpret_cast<const char *>(a.w) + pb;
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        load_row<Tin, PX>(P.u[r], bu, s.roff[r], s.col, last_col);
        load_row<Tin, PX>(P.v[r], bv, s.roff[r], s.col, last_col);
        load_row<Tin, PX>(P.w[r], bw, s.roff[r], s.col, last_col);
    }
    P.hu = Storage<Tin>::widen(*reinterpret_cast<const Tin *>(bu + s.hoff));
    P.hv = Storage<Tin>::widen(*reinterpret_cast<const Tin *>(bv + s.hoff));
    P.hw = Storage<Tin>::widen(*reinterpret_cast<const Tin *>(bw + s.hoff));
}

template <typename T, int N> __device__ __forceinline__ void store_vec(char *p, const T (&x)[N]) {
    typename Vec<T, N>::type v;
    if constexpr (N == 1) {
        v = x[0];
    } else {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = x[m];
    }
    __builtin_nontemporal_store(v, reinterpret_cast<typename Vec<T, N>::type *>(p));
}

// Source terms of output level kk (interior numbering) from planes kk-1 (m),
// kk (c) and kk+1 (p); stores the lanes/rows that own outputs.
template <typename Tin, int PX, int RY>
__device__ __forceinline__ void level(const Plane<typename Storage<Tin>::Tc, PX, RY> &m,
                                      const Plane<typename Storage<Tin>::Tc, PX, RY> &c,
                                      const Plane<typename Storage<Tin>::Tc, PX, RY> &p,
                                      const FwdK<Tin> &a, int kk, bool lane0, bool lane63, int nvalid,
                                      const uint32_t (&ooff)[RY], const bool (&row_ok)[RY]) {
    using Tc = typename Storage<Tin>::Tc;
    const Tc z1 = a.tzc1[kk], z2 = a.tzc2[kk], d1 = a.tzd1[kk], d2 = a.tzd2[kk];
    const Tc tcx = a.tcx, tcy = a.tcy;

    // Columns just outside this lane's PX columns, per loaded row, for the
    // arrays whose x-neighbours the stencil reads.
    Tc uL[RY + 2], uR[RY + 2], vL[RY + 2], vR[RY + 2], wL[RY + 2], wR[RY + 2], wRm[RY + 2], uLp[RY + 2];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        uL[r] = left_of(c.u[r][PX - 1], c.hu, r, lane0);
        uR[r] = right_of(c.u[r][0], c.hu, r, lane63);
        vL[r] = left_of(c.v[r][PX - 1], c.hv, r, lane0);
        vR[r] = right_of(c.v[r][0], c.hv, r, lane63);
        wL[r] = left_of(c.w[r][PX - 1], c.hw, r, lane0);
        wR[r] = right_of(c.w[r][0], c.hw, r, lane63);
        wRm[r] = right_of(m.w[r][0], m.hw, r, lane63);
        uLp[r] = left_of(p.u[r][PX - 1], p.hu, r, lane0);
    }
    // value at (row r, column x-1) / (row r, column x+1) of a plane array
#define XM(arr, L, r, x) ((x) == 0 ? L[r] : arr[r][(x) - 1])
#define XP(arr, R, r, x) ((x) == PX - 1 ? R[r] : arr[r][(x) + 1])

    // Face sums shared by consecutive rows of the strip (index r = loaded row):
    //   fy = v(k,r,i) + v(k,r,i+1)   gy = v(k,r,i) + v(k,r+1,i)   hy = v(k,r,i) + v(k+1,r,i)
    Tc fy[RY + 1][PX], gy[RY + 1][PX], hy[RY + 1][PX];
#pragma unroll
    for (int r = 0; r <= RY; ++r) {
#pragma unroll
        for (int x = 0; x < PX; ++x) {
            fy[r][x] = c.v[r][x] + XP(c.v, vR, r, x);
            gy[r][x] = c.v[r][x] + c.v[r + 1][x];
            hy[r][x] = c.v[r][x] + p.v[r][x];
        }
    }

    const int64_t ob = static_cast<int64_t>(kk) * a.out_sz * static_cast<int64_t>(sizeof(Tc));
    char *osu = reinterpret_cast<char *>(a.su) + ob;
    char *osv = reinterpret_cast<char *>(a.sv) + ob;
    char *osw = reinterpret_cast<char *>(a.sw) + ob;

#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int q = r + 1;   // this output row within the loaded rows
        Tc rsu[PX], rsv[PX], rsw[PX];
#pragma unroll
        for (int x = 0; x < PX; ++x) {
            // su: x faces (u+u), y faces (v+v at i, i+1), z faces (w+w at i, i+1)
            const Tc uc = c.u[q][x];
            const Tc ul = XM(c.u, uL, q, x), ur = XP(c.u, uR, q, x);
            const Tc ax = fma_(-ur, uc + ur, ul * (uc + ul));
            const Tc ay = fma_(-c.u[q + 1][x], fy[q][x], c.u[q - 1][x] * fy[r][x]);
            const Tc fzm = m.w[q][x] + XP(m.w, wRm, q, x);
            const Tc fzp = c.w[q][x] + XP(c.w, wR, q, x);
            Tc su = tcx * ax;
            su = fma_(tcy, ay, su);
            su = fma_(z1 * m.u[q][x], fzm, su);
            su = fma_(-(z2 * p.u[q][x]), fzp, su);

            // sv: x faces (u+u at j, j+1), y faces (v+v), z faces (w+w at j, j+1)
            const Tc vl = XM(c.v, vL, q, x), vr = XP(c.v, vR, q, x);
            const Tc gxp = uc + c.u[q + 1][x];
            const Tc gxm = ul + XM(c.u, uL, q + 1, x);
            const Tc bx = fma_(-vr, gxp, vl * gxm);
            const Tc by = fma_(-c.v[q + 1][x], gy[q][x], c.v[q - 1][x] * gy[r][x]);
            const Tc gzm = m.w[q][x] + m.w[q + 1][x];
            const Tc gzp = c.w[q][x] + c.w[q + 1][x];
            Tc sv = tcx * bx;
            sv = fma_(tcy, by, sv);
            sv = fma_(z1 * m.v[q][x], gzm, sv);
            sv = fma_(-(z2 * p.v[q][x]), gzp, sv);

            // sw: x faces (u+u at k, k+1), y faces (v+v at k, k+1), z faces (w+w)
            const Tc wc = c.w[q][x];
            const Tc wl = XM(c.w, wL, q, x), wr = XP(c.w, wR, q, x);
            const Tc hxp = uc + p.u[q][x];
            const Tc hxm = ul + XM(p.u, uLp, q, x);
            const Tc cx = fma_(-wr, hxp, wl * hxm);
            const Tc cy = fma_(-c.w[q + 1][x], hy[q][x], c.w[q - 1][x] * hy[r][x]);
            const Tc hzm = wc + m.w[q][x];
            const Tc hzp = wc + p.w[q][x];
            Tc sw = tcx * cx;
            sw = fma_(tcy, cy, sw);
            sw = fma_(d1 * m.w[q][x], hzm, sw);
            sw = fma_(-(d2 * p.w[q][x]), hzp, sw);

            rsu[x] = su;
            rsv[x] = sv;
            rsw[x] = sw;
        }
        if (row_ok[r]) {
            if (nvalid >= PX) {
                store_vec<Tc, PX>(osu + ooff[r], rsu);
                store_vec<Tc, PX>(osv + ooff[r], rsv);
                store_vec<Tc, PX>(osw + ooff[r], rsw);
            } else {
#pragma unroll
                for (int x = 0; x < PX; ++x) {
                    if (x < nvalid) {
                        __builtin_nontemporal_store(rsu[x], reinterpret_cast<Tc *>(osu + ooff[r]) + x);
                        __builtin_nontemporal_store(rsv[x], reinterpret_cast<Tc *>(osv + ooff[r]) + x);
                        __builtin_nontemporal_store(rsw[x], reinterpret_cast<Tc *>(osw + ooff[r]) + x);
                    }
                }
            }
        }
    }
#undef XM
#undef XP
}

// Workgroup -> tile numbering.  Workgroups are handed to the 8 XCDs round
// robin; give XCD x the contiguous tile range [start(x), start(x+1)).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, rem) + i;
}

template <typename Tin, int PX, int RY>
__global__ __launch_bounds__(512) void pw_forward_kernel(FwdK<Tin> a) {
    using Tc = typename Storage<Tin>::Tc;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cz = t % a.nzc;
    const int t2 = t / a.nzc;
    const int tx = t2 % a.ntx;
    const int ty = (t2 / a.ntx) * a.wpb + wave;
    if (ty >= a.nty) return;   // whole wavefront

    const int pcols = a.nx + 2 * a.h, prows = a.ny + 2 * a.h;
    const int last_col = pcols - 1;
    const int ii0 = tx * 64 * PX + lane * PX;        // first interior column of this lane
    const int nvalid = a.nx - ii0;                    // its columns inside the grid (may be <= 0)
    const int jj0 = ty * RY;

    StripAddr<RY> s;
    s.col = min(ii0 + a.h, last_col);
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int prow = min(jj0 - 1 + a.h + r, prows - 1);
        s.roff[r] = static_cast<uint32_t>((prow * a.in_sy + s.col) * static_cast<int>(sizeof(Tin)));
    }
    {   // packed halo: lane r -> left halo of row r, lane 32+r -> right halo of row r
        const int hr = min(lane & 31, RY + 1);
        const int hrow = min(jj0 - 1 + a.h + hr, prows - 1);
        const int hcol = (lane & 32) ? min(tx * 64 * PX + 64 * PX + a.h, last_col) : tx * 64 * PX + a.h - 1;
        s.hoff = static_cast<uint32_t>((hrow * a.in_sy + hcol) * static_cast<int>(sizeof(Tin)));
    }
    uint32_t ooff[RY];
    bool row_ok[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row_ok[r] = jj0 + r < a.ny;
        const int jj = min(jj0 + r, a.ny - 1);
        const int ic = min(ii0, a.nx - 1);
        ooff[r] = static_cast<uint32_t>((jj * a.out_sy + ic) * static_cast<int>(sizeof(Tc)));
    }
    const bool lane0 = lane == 0, lane63 = lane == 63;

    const int k0 = cz * a.zlen;
    const int k1 = min(a.nz, k0 + a.zlen);
    const int h = a.h;

    Plane<Tc, PX, RY> A, B, C, D;
    load_plane<Tin, PX, RY>(A, a, k0 - 1 + h, s, last_col);
    load_plane<Tin, PX, RY>(B, a, k0 + h, s, last_col);
    load_plane<Tin, PX, RY>(C, a, k0 + 1 + h, s, last_col);
    int kk = k0;
    for (;;) {
        if (kk + 1 < k1) load_plane<Tin, PX, RY>(D, a, kk + 2 + h, s, last_col);
        level<Tin, PX, RY>(A, B, C, a, kk, lane0, lane63, nvalid, ooff, row_ok);
        if (++kk >= k1) break;
        if (kk + 1 < k1) load_plane<Tin, PX, RY>(A, a, kk + 2 + h, s, last_col);
        level<Tin, PX, RY>(B, C, D, a, kk, lane0, lane63, nvalid, ooff, row_ok);
        if (++kk >= k1) break;
        if (kk + 1 < k1) load_plane<Tin, PX, RY>(B, a, kk + 2 + h, s, last_col);
        level<Tin, PX, RY>(C, D, A, a, kk, lane0, lane63, nvalid, ooff, row_ok);
        if (++kk >= k1) break;
        if (kk + 1 < k1) load_plane<Tin, PX, RY>(C, a, kk + 2 + h, s, last_col);
        level<Tin, PX, RY>(D, A, B, a, kk, lane0, lane63, nvalid, ooff, row_ok);
        if (++kk >= k1) break;
    }
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
    hipLaunchKernelGGL((pw_forward_kernel<Tin, PX, RY>), dim3(static_cast<unsigned>(nblocks)),
                       dim3(64 * cfg.wpb), 0, s, a);
    return hip_fail(hipGetLastError(), "forward kernel launch");
}

template <typename Tin, int PX>
pw_status launch_fwd_px(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.ry) {
        case 1: return launch_fwd_t<Tin, PX, 1>(g, cfg, s);
        case 2: return launch_fwd_t<Tin, PX, 2>(g, cfg, s);
        case 4:
            if constexpr (sizeof(Tin) <= 4 && PX <= 2) return launch_fwd_t<Tin, PX, 4>(g, cfg, s);
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

}  // namespace

bool tile_supported(const TileCfg &c, pw_dtype dt) {
    if (c.zlen < 1 || c.wpb < 1 || c.wpb > 8) return false;
    if (dt == PW_F64) return (c.px == 1 || c.px == 2) && (c.ry == 1 || c.ry == 2);
    if (c.px == 4) return c.ry == 1 || c.ry == 2;
    return (c.px == 1 || c.px == 2) && (c.ry == 1 || c.ry == 2 || c.ry == 4);
}

TileCfg default_forward_tile(const FwdArgs &a, pw_dtype dt) {
    // Measured on MI355X: one column per lane with two-row strips and four
    // strips per workgroup is the fastest family for FP32, FP64 and 16-bit
    // storage on the dense halo-padded layout; the march is cut into at least
    // two z-chunks, more when the grid has too few strips to give every CU
    // about 16 wavefronts.
    TileCfg c;
    c.px = 1;
    c.ry = 2;
    c.wpb = 4;
    (void)dt;
    const int64_t strips = ((a.nx + 63) / 64) * ((a.ny + c.ry - 1) / c.ry);
    int64_t chunks = (256 * 16 + strips - 1) / strips;
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
