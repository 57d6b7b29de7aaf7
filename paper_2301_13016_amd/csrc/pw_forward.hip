// Forward Piacsek-Williams advection kernel for gfx950 (CDNA4).
//
// What it computes: the source terms su, sv, sw of the PW scheme (paper
// Sec. 2.2; per-cell arithmetic of Sec. 4 / Fig. 2: six face sums, six
// products with a neighbouring value, signed reduction, same arithmetic for
// the three fields).  The equations are written out in include/pwadv.h.
//
// How (one wavefront = one independent work item, no LDS, no barriers):
//   * A wavefront owns a strip of 62 output columns x RY output rows and
//     marches upward through a chunk of z-levels.  Its 64 lanes load 64
//     consecutive padded columns, so the x-neighbours (i-1, i+1) of the 62
//     inner lanes are one lane away and come from DPP wavefront shifts that
//     the compiler folds into the consuming VALU instruction.
//   * Each lane keeps RY+2 rows (the strip plus one halo row above and below)
//     of u, v, w for four consecutive z-planes in registers: planes k-1, k,
//     k+1 feed the stencil at level k while plane k+2 is in flight.  The ring
//     is rotated by unrolling the march four ways, so no register moves.
//   * Every padded input element is fetched by one strip per z-chunk (plus
//     the strips' halo rows / columns, which neighbouring strips on the same
//     XCD fetch at about the same time and so hit L2).  Outputs are written
//     once with non-temporal stores.
//   * Workgroups are re-numbered so that each XCD (8 per MI355X, each with its
//     own L2) gets one contiguous range of tiles, ordered z-chunk fastest:
//     tiles that share halo planes and rows run on the same L2.
//
// Storage types: float, double, BF16 (uint16_t bit patterns) and FP16
// (_Float16).  16-bit values are widened exactly to float as they arrive;
// the arithmetic is float (double for double storage).
#include "pw_internal.h"

namespace pw {
namespace {

// ----------------------------------------------------------------- widening
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

// ------------------------------------------------------- wavefront shifts
// DPP controls (GFX9 family): wave_shr:1 moves lane l-1 into lane l,
// wave_shl:1 moves lane l+1 into lane l.  bound_ctrl makes the lane that has no
// source read 0; those edge lanes never store.
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
// value at column i-1 / i+1 of the lane's own column i
template <typename T> __device__ __forceinline__ T from_left(T x) { return wave_shift<kWaveShr1>(x); }
template <typename T> __device__ __forceinline__ T from_right(T x) { return wave_shift<kWaveShl1>(x); }

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
// jj0-1 .. jj0+RY (interior numbering), in this lane's column.
template <typename Tc, int RY> struct Plane {
    Tc u[RY + 2], v[RY + 2], w[RY + 2];
};

template <typename Tin, int RY>
__device__ __forceinline__ void load_plane(Plane<typename Storage<Tin>::Tc, RY> &P, const FwdK<Tin> &a,
                                           int kp, const uint32_t (&roff)[RY + 2]) {
    const int64_t pb = static_cast<int64_t>(kp) * a.in_sz * static_cast<int64_t>(sizeof(Tin));
    const char *bu = reinterpret_cast<const char *>(a.u) + pb;
    const char *bv = reinterpret_cast<const char *>(a.v) + pb;
    const char *bw = reinterpret_cast<const char *>(a.w) + pb;
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        P.u[r] = Storage<Tin>::widen(*reinterpret_cast<const Tin *>(bu + roff[r]));
        P.v[r] = Storage<Tin>::widen(*reinterpret_cast<const Tin *>(bv + roff[r]));
        P.w[r] = Storage<Tin>::widen(*reinterpret_cast<const Tin *>(bw + roff[r]));
    }
}

// Source terms of output level kk (interior numbering) from planes kk-1 (m),
// kk (c) and kk+1 (p); stores the lanes/rows that own an output.
template <typename Tin, int RY>
__device__ __forceinline__ void level(const Plane<typename Storage<Tin>::Tc, RY> &m,
                                      const Plane<typename Storage<Tin>::Tc, RY> &c,
                                      const Plane<typename Storage<Tin>::Tc, RY> &p,
                                      const FwdK<Tin> &a, int kk, bool lane_ok,
                                      const uint32_t (&ooff)[RY], const bool (&row_ok)[RY]) {
    using Tc = typename Storage<Tin>::Tc;
    const Tc z1 = a.tzc1[kk], z2 = a.tzc2[kk], d1 = a.tzd1[kk], d2 = a.tzd2[kk];
    const Tc tcx = a.tcx, tcy = a.tcy;

    // Face sums shared by consecutive rows of the strip (row r of these
    // arrays belongs to strip row r, i.e. interior row jj0-1+r):
    //   fy[r] = v(k,r,i) + v(k,r,i+1)    north face of the u cell below row r+1
    //   gy[r] = v(k,r,i) + v(k,r+1,i)    y face of the v cell
    //   hy[r] = v(k,r,i) + v(k+1,r,i)    north face of the w cell
    Tc fy[RY + 1], gy[RY + 1], hy[RY + 1];
#pragma unroll
    for (int r = 0; r <= RY; ++r) {
        fy[r] = c.v[r] + from_right(c.v[r]);
        gy[r] = c.v[r] + c.v[r + 1];
        hy[r] = c.v[r] + p.v[r];
    }

    const int64_t ob = static_cast<int64_t>(kk) * a.out_sz * static_cast<int64_t>(sizeof(Tc));
    char *osu = reinterpret_cast<char *>(a.su) + ob;
    char *osv = reinterpret_cast<char *>(a.sv) + ob;
    char *osw = reinterpret_cast<char *>(a.sw) + ob;

#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int q = r + 1;   // this output row within the loaded rows

        // su: x faces (u+u), y faces (v+v at i, i+1), z faces (w+w at i, i+1)
        const Tc ul = from_left(c.u[q]), ur = from_right(c.u[q]);
        const Tc ax = fma_(-ur, c.u[q] + ur, ul * (c.u[q] + ul));
        const Tc ay = fma_(-c.u[q + 1], fy[q], c.u[q - 1] * fy[r]);
        const Tc fzm = m.w[q] + from_right(m.w[q]);
        const Tc fzp = c.w[q] + from_right(c.w[q]);
        Tc su = tcx * ax;
        su = fma_(tcy, ay, su);
        su = fma_(z1 * m.u[q], fzm, su);
        su = fma_(-(z2 * p.u[q]), fzp, su);

        // sv: x faces (u+u at j, j+1), y faces (v+v), z faces (w+w at j, j+1)
        const Tc vl = from_left(c.v[q]), vr = from_right(c.v[q]);
        const Tc gxp = c.u[q] + c.u[q + 1];
        const Tc gxm = from_left(gxp);
        const Tc bx = fma_(-vr, gxp, vl * gxm);
        const Tc by = fma_(-c.v[q + 1], gy[q], c.v[q - 1] * gy[r]);
        const Tc gzm = m.w[q] + m.w[q + 1];
        const Tc gzp = c.w[q] + c.w[q + 1];
        Tc sv = tcx * bx;
        sv = fma_(tcy, by, sv);
        sv = fma_(z1 * m.v[q], gzm, sv);
        sv = fma_(-(z2 * p.v[q]), gzp, sv);

        // sw: x faces (u+u at k, k+1), y faces (v+v at k, k+1), z faces (w+w)
        const Tc wl = from_left(c.w[q]), wr = from_right(c.w[q]);
        const Tc hxp = c.u[q] + p.u[q];
        const Tc hxm = from_left(hxp);
        const Tc cx = fma_(-wr, hxp, wl * hxm);
        const Tc cy = fma_(-c.w[q + 1], hy[q], c.w[q - 1] * hy[r]);
        const Tc hzm = c.w[q] + m.w[q];
        const Tc hzp = c.w[q] + p.w[q];
        Tc sw = tcx * cx;
        sw = fma_(tcy, cy, sw);
        sw = fma_(d1 * m.w[q], hzm, sw);
        sw = fma_(-(d2 * p.w[q]), hzp, sw);

        if (lane_ok && row_ok[r]) {
            __builtin_nontemporal_store(su, reinterpret_cast<Tc *>(osu + ooff[r]));
            __builtin_nontemporal_store(sv, reinterpret_cast<Tc *>(osv + ooff[r]));
            __builtin_nontemporal_store(sw, reinterpret_cast<Tc *>(osw + ooff[r]));
        }
    }
}

// Workgroup -> tile numbering.  Workgroups are handed to the 8 XCDs round
// robin; give XCD x the contiguous tile range [start(x), start(x+1)).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, rem) + i;
}

template <typename Tin, int RY>
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

    // Columns: lane l loads padded column tx*62 + h-1 + l (clamped into the
    // array; clamped lanes never own an output).
    const int pcols = a.nx + 2 * a.h, prows = a.ny + 2 * a.h;
    const int col = min(tx * kWaveCols + a.h - 1 + lane, pcols - 1);
    const int ii = tx * kWaveCols + lane - 1;             // interior column owned
    const bool lane_ok = lane >= 1 && lane <= kWaveCols && ii < a.nx;
    const int jj0 = ty * RY;

    uint32_t roff[RY + 2];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int prow = min(jj0 - 1 + a.h + r, prows - 1);
        roff[r] = static_cast<uint32_t>((prow * a.in_sy + col) * static_cast<int>(sizeof(Tin)));
    }
    uint32_t ooff[RY];
    bool row_ok[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row_ok[r] = jj0 + r < a.ny;
        const int jj = min(jj0 + r, a.ny - 1);
        const int ic = min(max(ii, 0), a.nx - 1);
        ooff[r] = static_cast<uint32_t>((jj * a.out_sy + ic) * static_cast<int>(sizeof(Tc)));
    }

    const int k0 = cz * a.zlen;
    const int k1 = min(a.nz, k0 + a.zlen);
    const int h = a.h;

    Plane<Tc, RY> A, B, C, D;
    load_plane<Tin, RY>(A, a, k0 - 1 + h, roff);
    load_plane<Tin, RY>(B, a, k0 + h, roff);
    load_plane<Tin, RY>(C, a, k0 + 1 + h, roff);
    int kk = k0;
    for (;;) {
        if (kk + 1 < k1) load_plane<Tin, RY>(D, a, kk + 2 + h, roff);
        level<Tin, RY>(A, B, C, a, kk, lane_ok, ooff, row_ok);
        if (++kk >= k1) break;
        if (kk + 1 < k1) load_plane<Tin, RY>(A, a, kk + 2 + h, roff);
        level<Tin, RY>(B, C, D, a, kk, lane_ok, ooff, row_ok);
        if (++kk >= k1) break;
        if (kk + 1 < k1) load_plane<Tin, RY>(B, a, kk + 2 + h, roff);
        level<Tin, RY>(C, D, A, a, kk, lane_ok, ooff, row_ok);
        if (++kk >= k1) break;
        if (kk + 1 < k1) load_plane<Tin, RY>(C, a, kk + 2 + h, roff);
        level<Tin, RY>(D, A, B, a, kk, lane_ok, ooff, row_ok);
        if (++kk >= k1) break;
    }
}

template <typename Tin, int RY>
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
    a.ntx = static_cast<int32_t>((g.nx + kWaveCols - 1) / kWaveCols);
    a.nty = static_cast<int32_t>((g.ny + RY - 1) / RY);
    a.zlen = cfg.zlen;
    a.nzc = static_cast<int32_t>((g.nz + cfg.zlen - 1) / cfg.zlen);
    a.wpb = cfg.wpb;
    const int64_t nblk_y = (a.nty + cfg.wpb - 1) / cfg.wpb;
    const int64_t nblocks = static_cast<int64_t>(a.ntx) * nblk_y * a.nzc;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    hipLaunchKernelGGL((pw_forward_kernel<Tin, RY>), dim3(static_cast<unsigned>(nblocks)),
                       dim3(64 * cfg.wpb), 0, s, a);
    return hip_fail(hipGetLastError(), "forward kernel launch");
}

template <typename Tin>
pw_status launch_fwd_dt(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    switch (cfg.ry) {
        case 1: return launch_fwd_t<Tin, 1>(g, cfg, s);
        case 2: return launch_fwd_t<Tin, 2>(g, cfg, s);
        case 4: return launch_fwd_t<Tin, 4>(g, cfg, s);
        case 8:
            if constexpr (sizeof(Tin) <= 4) return launch_fwd_t<Tin, 8>(g, cfg, s);
            [[fallthrough]];
        default: return fail(PW_ERR_UNSUPPORTED, "rows per strip %d not instantiated", cfg.ry);
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

bool tile_supported(const TileCfg &c) {
    return (c.ry == 1 || c.ry == 2 || c.ry == 4 || c.ry == 8) && c.zlen >= 1 && c.wpb >= 1 && c.wpb <= 8;
}

TileCfg default_forward_tile(const FwdArgs &a, pw_dtype dt) {
    TileCfg c;
    c.ry = (dt == PW_F64) ? 2 : 4;
    c.wpb = 4;
    // Enough independent wavefronts to fill 256 CUs several times over, but
    // long enough marches that the two re-read planes per chunk stay cheap.
    const int64_t strips = ((a.nx + kWaveCols - 1) / kWaveCols) * ((a.ny + c.ry - 1) / c.ry);
    const int64_t want = 256 * 24;
    int64_t chunks = (want + strips - 1) / strips;
    if (chunks < 1) chunks = 1;
    int64_t zl = (a.nz + chunks - 1) / chunks;
    if (zl < 8) zl = 8;
    if (zl > a.nz) zl = a.nz;
    c.zlen = static_cast<int>(zl);
    return c;
}

pw_status launch_forward(const FwdArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s) {
    if (!tile_supported(cfg)) return fail(PW_ERR_INVALID_ARG, "unsupported tile configuration");
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
