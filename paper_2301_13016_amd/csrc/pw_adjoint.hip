// Adjoint (vector-Jacobian product) of the PW advection operator, gfx950.
//
// Given output cotangents (gsu, gsv, gsw) on the interior, computes
//   (gu, gv, gw) = J(u, v, w)^T (gsu, gsv, gsw)
// on the whole padded grid (halo included), in gather form: each gradient
// point q collects, from the outputs p whose product terms read q, the partial
// derivative of that term times the cotangent at p.  A term
//   s * c * a * (b + d)
// contributes s*c*(b+d)*r to the gradient of a and s*c*a*r to those of b and d
// (product rule); writing q's contributions grouped by cotangent point gives
// the expressions below (15 cotangent points per gradient point, all within
// one cell in every direction).  No atomics: every gradient entry is written
// by exactly one lane.
//
// Layout and launch mirror the forward kernel: a wavefront owns a strip of 62
// padded columns x RY padded rows and marches through padded z-levels with a
// four-plane register ring (values u, v, w and cotangents of planes k-1, k,
// k+1 feed level k while k+2 is in flight); x-neighbours come from DPP
// wavefront shifts.  Cotangents outside the interior read as 0.  Values in
// cells that no output reads (3-D halo corners, most halo edges, every cell
// beyond the first halo layer, and positions outside the padded array, which
// are loaded from the nearest valid entry) read as 0 as well: they only ever
// meet zero cotangents, and zeroing them keeps a non-finite value there
// (0 * NaN = NaN) out of the gradient.
#include "pw_internal.h"
#include "pw_lanes.h"
#include "pw_reduce.h"

namespace pw {
namespace {

using lanes::fma_;
using lanes::kWaveShl1;
using lanes::kWaveShr1;
using lanes::wave_shift;
template <typename T> __device__ __forceinline__ T from_left(T x) { return wave_shift<kWaveShr1>(x); }   // lane l-1
template <typename T> __device__ __forceinline__ T from_right(T x) { return wave_shift<kWaveShl1>(x); }  // lane l+1

template <typename T> struct AdjK {
    const T *u, *v, *w;
    const T *ru, *rv, *rw;          // cotangents of su, sv, sw (interior, output layout)
    T *gu, *gv, *gw;                // gradients (padded, input layout)
    const T *tzc1, *tzc2, *tzd1, *tzd2;
    T tcx, tcy;
    int32_t nx, ny, nz, h;
    int64_t in_sz, out_sz;
    int32_t in_sy, out_sy;
    int32_t ntx, nty, nzc, zlen, wpb;
    // coefficient partials (modes with kModeCg): ws[q][level][strip], strip = ty * ntx + tx
    double *ws;
};

// What a launch computes: the gradients of u, v, w (kModeGrad), the
// per-strip coefficient partials (kModeCg; see cg_level), or both in one pass.
constexpr int kModeGrad = 1, kModeCg = 2;

// One padded z-plane of the strip: rows 0..RY+1 are padded rows jb-1 .. jb+RY.
template <typename T, int RY> struct APlane {
    T u[RY + 2], v[RY + 2], w[RY + 2];
    T ru[RY + 2], rv[RY + 2], rw[RY + 2];
    bool zok;   // the plane is an interior level, so its cotangents exist (wave-uniform)
    int kcls;   // position class of the plane (wave-uniform), see pos_class
};

// Bits of StripAddr::mask for one loaded row and the lane's column: bit
// 3*kc + f (f = 0, 1, 2 for u, v, w) is set when the forward operator reads
// that field's cell on a plane of position class kc; kCotOk is set when the
// row and column are inside the interior (its cotangent exists).
constexpr uint32_t kCotOk = 1u << 12;

template <typename T, int RY> struct StripAddr {
    uint32_t voff[RY + 2];   // byte offsets of the value rows (clamped)
    uint32_t roff[RY + 2];   // byte offsets of the cotangent rows (clamped)
    uint32_t mask[RY + 2];   // per row, see kCotOk
};

// Position class of a padded coordinate x along an axis with interior
// [h, h + n): 0 interior, 1 the halo layer just below it, 2 the layer just
// above it, 3 anything further out (including outside the padded array).
__device__ __forceinline__ int pos_class(int x, int h, int n) {
    return (x >= h && x < h + n) ? 0 : (x == h - 1) ? 1 : (x == h + n) ? 2 : 3;
}

// Whether the forward operator reads a cell of u, v or w, from the classes
// of its k, j, i coordinates.  Each output reads its point's 7-point star of
// every field plus two diagonal neighbours per field (u at (0,+1,-1) and
// (+1,0,-1), v at (0,-1,+1) and (+1,-1,0), w at (-1,0,+1) and (-1,+1,0));
// so a cell is read when it is inside or in the first halo layer of one
// axis, or when it sits on the one halo edge per diagonal that such a
// neighbour reaches.
__device__ __forceinline__ void cells_read(int kc, int jc, int ic, bool &ru_, bool &rv_, bool &rw_) {
    const bool far = kc == 3 || jc == 3 || ic == 3;
    const bool star = (kc != 0) + (jc != 0) + (ic != 0) <= 1;
    const int code = kc * 16 + jc * 4 + ic;
    ru_ = !far && (star || code == 0 * 16 + 2 * 4 + 1 || code == 2 * 16 + 0 * 4 + 1);
    rv_ = !far && (star || code == 0 * 16 + 1 * 4 + 2 || code == 2 * 16 + 1 * 4 + 0);
    rw_ = !far && (star || code == 1 * 16 + 0 * 4 + 2 || code == 1 * 16 + 2 * 4 + 0);
}

// Buffer descriptor of one z-plane (base: the plane; range: its bytes, below
// 2 GiB; word 3 as the GFX9 family wants it for untyped access).  Loads and
// stores then take the row offset as a 32-bit offset and need no 64-bit
// address arithmetic per access; an offset past the range would read 0 and
// drop a write.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, static_cast<int>(bytes), 0x00020000);
}
template <typename T> __device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <typename T> __device__ __forceinline__ void bstore(T x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, off, 0, 0);
    } else {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, off, 0, 0);
    }
}

template <typename T, int RY>
__device__ __forceinline__ void load_aplane(APlane<T, RY> &P, const AdjK<T> &a, int kp, const StripAddr<T, RY> &s) {
    const int pz = a.nz + 2 * a.h;
    const int kv = min(max(kp, 0), pz - 1);
    const int64_t pb = static_cast<int64_t>(kv) * a.in_sz * static_cast<int64_t>(sizeof(T));
    const int64_t vbytes = a.in_sz * static_cast<int64_t>(sizeof(T));
    const auto bu = plane_rsrc(reinterpret_cast<const char *>(a.u) + pb, vbytes);
    const auto bv = plane_rsrc(reinterpret_cast<const char *>(a.v) + pb, vbytes);
    const auto bw = plane_rsrc(reinterpret_cast<const char *>(a.w) + pb, vbytes);
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        P.u[r] = bload<T>(bu, s.voff[r]);
        P.v[r] = bload<T>(bv, s.voff[r]);
        P.w[r] = bload<T>(bw, s.voff[r]);
    }
    // Cotangents: every load from a clamped (valid) address and without a
    // branch, so that the plane's loads stay in flight until its first use,
    // where mask_aplane zeroes what lies outside the interior.
    const int kk = kp - a.h;
    P.zok = kk >= 0 && kk < a.nz;
    P.kcls = (kp < 0 || kp >= pz) ? 3 : pos_class(kp, a.h, a.nz);
    const int kc = min(max(kk, 0), a.nz - 1);
    const int64_t ob = static_cast<int64_t>(kc) * a.out_sz * static_cast<int64_t>(sizeof(T));
    const int64_t obytes = a.out_sz * static_cast<int64_t>(sizeof(T));
    const auto cu = plane_rsrc(reinterpret_cast<const char *>(a.ru) + ob, obytes);
    const auto cv = plane_rsrc(reinterpret_cast<const char *>(a.rv) + ob, obytes);
    const auto cw = plane_rsrc(reinterpret_cast<const char *>(a.rw) + ob, obytes);
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        P.ru[r] = bload<T>(cu, s.roff[r]);
        P.rv[r] = bload<T>(cv, s.roff[r]);
        P.rw[r] = bload<T>(cw, s.roff[r]);
    }
}

// Zero the cotangents of a loaded plane outside the interior, and the values
// of cells no output reads (once per plane, at its first use).
template <typename T, int RY>
__device__ __forceinline__ void mask_aplane(APlane<T, RY> &P, const StripAddr<T, RY> &s) {
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const bool ok = P.zok && (s.mask[r] & kCotOk);
        P.ru[r] = ok ? P.ru[r] : T(0);
        P.rv[r] = ok ? P.rv[r] : T(0);
        P.rw[r] = ok ? P.rw[r] : T(0);
        const uint32_t rd = s.mask[r] >> (3 * P.kcls);
        P.u[r] = (rd & 1u) ? P.u[r] : T(0);
        P.v[r] = (rd & 2u) ? P.v[r] : T(0);
        P.w[r] = (rd & 4u) ? P.w[r] : T(0);
    }
}

// Coefficient at a wave-uniform level, as a scalar load through the constant
// address space (the library rejects gradients that overlap the coefficient
// arrays); clamped: only ever met by a zero cotangent when outside.
template <typename T> __device__ __forceinline__ T coef(const T *c, int kk, int nz) {
    return ((const __attribute__((address_space(4))) T *)(c))[min(max(kk, 0), nz - 1)];
}

// Gradients at padded level kp from planes kp-1 (m), kp (c), kp+1 (p).
template <typename T, int RY>
__device__ __forceinline__ void adj_level(const APlane<T, RY> &m, const APlane<T, RY> &c, APlane<T, RY> &p,
                                          const AdjK<T> &a, const StripAddr<T, RY> &s, int kp, bool lane_ok,
                                          const uint32_t (&goff)[RY], const bool (&row_ok)[RY]) {
    const int kq = kp - a.h;   // interior level index of this gradient plane
    const T tcx = a.tcx, tcy = a.tcy;
    const T c1p = coef(a.tzc1, kq + 1, a.nz), c2m = coef(a.tzc2, kq - 1, a.nz), c2 = coef(a.tzc2, kq, a.nz);
    const T d1 = coef(a.tzd1, kq, a.nz), d2 = coef(a.tzd2, kq, a.nz);
    const T d2m = coef(a.tzd2, kq - 1, a.nz), d1p = coef(a.tzd1, kq + 1, a.nz);

    // Row-shared pieces (index r = loaded row r):
    //   xv[r] = rv(r,i+1) v(r,i) - rv(r,i) v(r,i+1)          plane k   (gu: sv x-terms)
    //   fy[r] = v(r,i) + v(r,i+1)                              plane k   (gu: su y-faces)
    //   hy[r] = v(k,r,i) + v(k+1,r,i)                                    (gw: sw y-faces)
    //   zv[r] = tzc1[kq+1] rv(k+1,r) v(k,r) - tzc2[kq] rv(k,r) v(k+1,r)  (gw: sv z-terms)
    T xv[RY + 1], fy[RY + 1], hy[RY + 1], zv[RY + 1];
#pragma unroll
    for (int r = 0; r <= RY; ++r) {
        xv[r] = fma_(from_right(c.rv[r]), c.v[r], -(c.rv[r] * from_right(c.v[r])));
        fy[r] = c.v[r] + from_right(c.v[r]);
        hy[r] = c.v[r] + p.v[r];
        zv[r] = fma_(c1p * p.rv[r], c.v[r], -(c2 * c.rv[r] * p.v[r]));
    }

    const int64_t gb = static_cast<int64_t>(min(max(kp, 0), a.nz + 2 * a.h - 1)) * a.in_sz *
                       static_cast<int64_t>(sizeof(T));
    const int64_t gbytes = a.in_sz * static_cast<int64_t>(sizeof(T));
    const auto ogu = plane_rsrc(reinterpret_cast<char *>(a.gu) + gb, gbytes);
    const auto ogv = plane_rsrc(reinterpret_cast<char *>(a.gv) + gb, gbytes);
    const auto ogw = plane_rsrc(reinterpret_cast<char *>(a.gw) + gb, gbytes);

#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int q = r + 1;
        const T two = T(2);

        // ---------------------------------------------------------------- gu
        const T ru_l = from_left(c.ru[q]), ru_r = from_right(c.ru[q]);
        const T u_l = from_left(c.u[q]), u_r = from_right(c.u[q]);
        // su x-terms
        T gx = ru_r * fma_(two, c.u[q], u_r);
        gx = fma_(c.ru[q], u_l - u_r, gx);
        gx = fma_(-ru_l, fma_(two, c.u[q], u_l), gx);
        // sv and sw x-terms: antisymmetric pairs at rows j-1, j (sv) and planes k-1, k (sw)
        const T xw_c = fma_(from_right(c.rw[q]), c.w[q], -(c.rw[q] * from_right(c.w[q])));
        const T xw_m = fma_(from_right(m.rw[q]), m.w[q], -(m.rw[q] * from_right(m.w[q])));
        gx = gx + ((xv[r] + xv[q]) + (xw_m + xw_c));
        // su y-terms
        const T gyu = fma_(c.ru[q + 1], fy[q], -(c.ru[q - 1] * fy[r]));
        // su z-terms
        const T gzu = fma_(c1p * p.ru[q], c.w[q] + from_right(c.w[q]),
                           -(c2m * m.ru[q] * (m.w[q] + from_right(m.w[q]))));
        T gu = tcx * gx;
        gu = fma_(tcy, gyu, gu);
        gu = gu + gzu;

        // ---------------------------------------------------------------- gv
        // su y-terms: yu(i) + yu(i-1), yu = ru(j+1) u(j) - ru(j) u(j+1)
        const T yu = fma_(c.ru[q + 1], c.u[q], -(c.ru[q] * c.u[q + 1]));
        const T gyv_su = yu + from_left(yu);
        // sv x-terms
        const T sxu = c.u[q] + c.u[q + 1];   // u(j,i) + u(j+1,i)
        const T gxv = fma_(from_right(c.rv[q]), sxu, -(from_left(c.rv[q]) * from_left(sxu)));
        // sv y-terms
        T gyv = c.rv[q + 1] * fma_(two, c.v[q], c.v[q + 1]);
        gyv = fma_(c.rv[q], c.v[q - 1] - c.v[q + 1], gyv);
        gyv = fma_(-c.rv[q - 1], fma_(two, c.v[q], c.v[q - 1]), gyv);
        // sw y-terms at planes k-1 and k: yw = rw(j+1) w(j) - rw(j) w(j+1)
        const T yw_c = fma_(c.rw[q + 1], c.w[q], -(c.rw[q] * c.w[q + 1]));
        const T yw_m = fma_(m.rw[q + 1], m.w[q], -(m.rw[q] * m.w[q + 1]));
        // sv z-terms
        const T gzv = fma_(c1p * p.rv[q], c.w[q] + c.w[q + 1], -(c2m * m.rv[q] * (m.w[q] + m.w[q + 1])));
        T gv = tcx * gxv;
        gv = fma_(tcy, (gyv_su + gyv) + (yw_m + yw_c), gv);
        gv = gv + gzv;

        // ---------------------------------------------------------------- gw
        // su z-terms: zu(i) + zu(i-1), zu = tzc1[kq+1] ru(k+1) u(k) - tzc2[kq] ru(k) u(k+1)
        const T zu = fma_(c1p * p.ru[q], c.u[q], -(c2 * c.ru[q] * p.u[q]));
        // sw z-terms
        T gzw = d1p * p.rw[q] * fma_(two, c.w[q], p.w[q]);
        gzw = fma_(c.rw[q], fma_(d1, m.w[q], -(d2 * p.w[q])), gzw);
        gzw = fma_(-(d2m * m.rw[q]), fma_(two, c.w[q], m.w[q]), gzw);
        // sw x-terms
        const T hxu = c.u[q] + p.u[q];   // u(k,i) + u(k+1,i)
        const T gxw = fma_(from_right(c.rw[q]), hxu, -(from_left(c.rw[q]) * from_left(hxu)));
        // sw y-terms
        const T gyw = fma_(c.rw[q + 1], hy[q], -(c.rw[q - 1] * hy[r]));
        T gw = (zu + from_left(zu)) + (zv[q] + zv[r]);
        gw = gw + gzw;
        gw = fma_(tcx, gxw, gw);
        gw = fma_(tcy, gyw, gw);

        if (lane_ok && row_ok[r]) {
            bstore<T>(gu, ogu, goff[r]);
            bstore<T>(gv, ogv, goff[r]);
            bstore<T>(gw, ogw, goff[r]);
        }
    }
}

// Coefficient partials of level kp (an interior level kk = kp - h): each
// coefficient multiplies a coefficient-free product in every term it enters,
// so dL/dc sums, over the interior points, the cotangent times that product.
// Per point the six groups (tzc1: z-lower u and v terms, tzc2: z-upper,
// tzd1 / tzd2: the w terms, tcx / tcy: the x- and y-face terms) are formed
// from the planes and rows the adjoint already holds, summed per lane over
// the strip's rows in the compute type, then over the wavefront in FP64 in a
// fixed order (red::wave_sum6), and stored as ws[q][kk][strip].  The strips are the adjoint's
// (62 columns x RY rows), so a partial does not depend on whether the
// gradients are computed in the same pass.  Points outside the interior, and
// lanes 0 and 63, are selected away (not multiplied by a zero cotangent: a
// NaN there would survive).
constexpr int kQ = 6;
template <typename T, int RY>
__device__ __forceinline__ void cg_level(const APlane<T, RY> &m, const APlane<T, RY> &c, const APlane<T, RY> &p,
                                         const AdjK<T> &a, const StripAddr<T, RY> &s, int kp, bool lane_ok,
                                         int strip) {
    if (!c.zok) return;   // a halo level (wave-uniform)
    T fy[RY + 1];
#pragma unroll
    for (int r = 0; r <= RY; ++r) fy[r] = c.v[r] + from_right(c.v[r]);
    T sq[kQ] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int q = r + 1;
        const bool ok = lane_ok && (s.mask[q] & kCotOk);
        const T ra = c.ru[q], rb = c.rv[q], re = c.rw[q];
        // su term groups
        const T uc = c.u[q], ul = from_left(c.u[q]), ur = from_right(c.u[q]);
        const T ax = fma_(-ur, uc + ur, ul * (uc + ul));
        const T ay = fma_(-c.u[q + 1], fy[q], c.u[q - 1] * fy[r]);
        const T az1 = m.u[q] * (m.w[q] + from_right(m.w[q]));
        const T az2 = p.u[q] * (c.w[q] + from_right(c.w[q]));
        // sv term groups
        const T vc = c.v[q], vl = from_left(c.v[q]), vr = from_right(c.v[q]);
        const T bx = fma_(-vr, uc + c.u[q + 1], vl * (ul + from_left(c.u[q + 1])));
        const T by = fma_(-c.v[q + 1], vc + c.v[q + 1], c.v[q - 1] * (vc + c.v[q - 1]));
        const T bz1 = m.v[q] * (m.w[q] + m.w[q + 1]);
        const T bz2 = p.v[q] * (c.w[q] + c.w[q + 1]);
        // sw term groups
        const T wc = c.w[q], wl = from_left(c.w[q]), wr = from_right(c.w[q]);
        const T cx = fma_(-wr, uc + p.u[q], wl * (ul + from_left(p.u[q])));
        const T cy = fma_(-c.w[q + 1], c.v[q] + p.v[q], c.w[q - 1] * (c.v[q - 1] + p.v[q - 1]));
        const T cz1 = m.w[q] * (wc + m.w[q]);
        const T cz2 = p.w[q] * (wc + p.w[q]);
        sq[0] += ok ? fma_(ra, az1, rb * bz1) : T(0);
        sq[1] -= ok ? fma_(ra, az2, rb * bz2) : T(0);
        sq[2] += ok ? re * cz1 : T(0);
        sq[3] -= ok ? re * cz2 : T(0);
        sq[4] += ok ? fma_(ra, ax, fma_(rb, bx, re * cx)) : T(0);
        sq[5] += ok ? fma_(ra, ay, fma_(rb, by, re * cy)) : T(0);
    }
    const int kk = kp - a.h;
    double qd[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) qd[q] = static_cast<double>(sq[q]);
    // one wavefront sum for all six (every lane ends with one quantity's total)
    const double t = red::wave_sum6(qd);
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int q = red::sum6_quantity(lane);
    if (lane < 8 && q < kQ)
        a.ws[(static_cast<int64_t>(q) * a.nz + kk) * (static_cast<int64_t>(a.ntx) * a.nty) + strip] = t;
}

__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, rem) + i;
}

// Depth: planes in flight ahead of the three a level reads (1 or 2).
// MaxT: workgroup size bound (built for 256 and 512 threads; see the forward
// kernel).
template <typename T, int RY, int Depth, int MaxT, int Mode>
__global__ __launch_bounds__(MaxT) void pw_adjoint_kernel(AdjK<T> a) {
    const int lane = threadIdx.x & 63;
    // wavefront index as a scalar, so that per-strip conditions stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cz = t % a.nzc;
    const int t2 = t / a.nzc;
    const int tx = t2 % a.ntx;
    const int ty = (t2 / a.ntx) * a.wpb + wave;
    if (ty >= a.nty) return;

    const int px = a.nx + 2 * a.h, py = a.ny + 2 * a.h, pz = a.nz + 2 * a.h;
    const int pcol = tx * kWaveCols - 1 + lane;        // padded column loaded by this lane
    const int vcol = min(max(pcol, 0), px - 1);
    const int icol = pcol - a.h;                        // its interior column
    const bool lane_ok = lane >= 1 && lane <= kWaveCols && pcol < px;
    const int jb = ty * RY;                             // first padded gradient row

    StripAddr<T, RY> s;
    const bool rcol = icol >= 0 && icol < a.nx;
    const int icls = (pcol < 0 || pcol >= px) ? 3 : pos_class(pcol, a.h, a.nx);
    const int icl = min(max(icol, 0), a.nx - 1);
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int prow = jb - 1 + r;
        const int vr = min(max(prow, 0), py - 1);
        s.voff[r] = static_cast<uint32_t>((vr * a.in_sy + vcol) * static_cast<int>(sizeof(T)));
        const int ir = prow - a.h;
        const int jcls = (prow < 0 || prow >= py) ? 3 : pos_class(prow, a.h, a.ny);
        uint32_t m = (rcol && ir >= 0 && ir < a.ny) ? kCotOk : 0u;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            bool read_u, read_v, read_w;
            cells_read(kc, jcls, icls, read_u, read_v, read_w);
            m |= (read_u ? 1u : 0u) << (3 * kc);
            m |= (read_v ? 2u : 0u) << (3 * kc);
            m |= (read_w ? 4u : 0u) << (3 * kc);
        }
        s.mask[r] = m;
        const int irc = min(max(ir, 0), a.ny - 1);
        s.roff[r] = static_cast<uint32_t>((irc * a.out_sy + icl) * static_cast<int>(sizeof(T)));
    }
    uint32_t goff[RY];
    bool row_ok[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row_ok[r] = jb + r < py;
        const int gr = min(jb + r, py - 1);
        goff[r] = static_cast<uint32_t>((gr * a.in_sy + vcol) * static_cast<int>(sizeof(T)));
    }

    const int k0 = cz * a.zlen;
    const int k1 = min(pz, k0 + a.zlen);
    // Unconditional prefetch (past the chunk's last level it re-reads plane
    // k1, a cache hit, into a slot no level uses): a conditional load would
    // join two paths with different loads in flight, and the wait at the join
    // drains the prefetch.
    const int strip = ty * a.ntx + tx;
#define PW_ALEVEL(M, C, P)                                                                    \
    do {                                                                                      \
        mask_aplane<T, RY>(P, s);   /* first use of plane k+1 */                              \
        if constexpr (Mode & kModeGrad) adj_level<T, RY>(M, C, P, a, s, k, lane_ok, goff, row_ok); \
        if constexpr (Mode & kModeCg) cg_level<T, RY>(M, C, P, a, s, k, lane_ok, strip);           \
    } while (0)
    int k = k0;
    if constexpr (Depth == 1) {
        // four-plane ring: planes k-1, k, k+1 feed level k, k+2 in flight
        APlane<T, RY> A, B, C, D;
        load_aplane<T, RY>(A, a, k0 - 1, s);
        load_aplane<T, RY>(B, a, k0, s);
        load_aplane<T, RY>(C, a, k0 + 1, s);
        mask_aplane<T, RY>(A, s);
        mask_aplane<T, RY>(B, s);
        for (;;) {
            load_aplane<T, RY>(D, a, min(k + 2, k1), s);
            PW_ALEVEL(A, B, C);
            if (++k >= k1) break;
            load_aplane<T, RY>(A, a, min(k + 2, k1), s);
            PW_ALEVEL(B, C, D);
            if (++k >= k1) break;
            load_aplane<T, RY>(B, a, min(k + 2, k1), s);
            PW_ALEVEL(C, D, A);
            if (++k >= k1) break;
            load_aplane<T, RY>(C, a, min(k + 2, k1), s);
            PW_ALEVEL(D, A, B);
            if (++k >= k1) break;
        }
    } else {
        // five-plane ring: planes k+2 and k+3 in flight
        static_assert(Depth == 2, "prefetch depth 1 or 2");
        APlane<T, RY> A, B, C, D, E;
        load_aplane<T, RY>(A, a, k0 - 1, s);
        load_aplane<T, RY>(B, a, k0, s);
        load_aplane<T, RY>(C, a, k0 + 1, s);
        load_aplane<T, RY>(D, a, min(k0 + 2, k1), s);
        mask_aplane<T, RY>(A, s);
        mask_aplane<T, RY>(B, s);
        for (;;) {
            load_aplane<T, RY>(E, a, min(k + 3, k1), s);
            PW_ALEVEL(A, B, C);
            if (++k >= k1) break;
            load_aplane<T, RY>(A, a, min(k + 3, k1), s);
            PW_ALEVEL(B, C, D);
            if (++k >= k1) break;
            load_aplane<T, RY>(B, a, min(k + 3, k1), s);
            PW_ALEVEL(C, D, E);
            if (++k >= k1) break;
            load_aplane<T, RY>(C, a, min(k + 3, k1), s);
            PW_ALEVEL(D, E, A);
            if (++k >= k1) break;
            load_aplane<T, RY>(D, a, min(k + 3, k1), s);
            PW_ALEVEL(E, A, B);
            if (++k >= k1) break;
        }
    }
#undef PW_ALEVEL
}

template <typename T, int RY, int Mode>
pw_status launch_adj_t(const AdjArgs &g, const TileCfg &cfg, double *ws, hipStream_t s) {
    AdjK<T> a;
    a.ws = ws;
    a.u = static_cast<const T *>(g.u);
    a.v = static_cast<const T *>(g.v);
    a.w = static_cast<const T *>(g.w);
    a.ru = static_cast<const T *>(g.gsu);
    a.rv = static_cast<const T *>(g.gsv);
    a.rw = static_cast<const T *>(g.gsw);
    a.gu = static_cast<T *>(g.gu);
    a.gv = static_cast<T *>(g.gv);
    a.gw = static_cast<T *>(g.gw);
    a.tzc1 = static_cast<const T *>(g.tzc1);
    a.tzc2 = static_cast<const T *>(g.tzc2);
    a.tzd1 = static_cast<const T *>(g.tzd1);
    a.tzd2 = static_cast<const T *>(g.tzd2);
    a.tcx = static_cast<T>(g.tcx);
    a.tcy = static_cast<T>(g.tcy);
    a.nx = static_cast<int32_t>(g.nx);
    a.ny = static_cast<int32_t>(g.ny);
    a.nz = static_cast<int32_t>(g.nz);
    a.h = g.h;
    a.in_sz = g.in_sz;
    a.out_sz = g.out_sz;
    a.in_sy = static_cast<int32_t>(g.in_sy);
    a.out_sy = static_cast<int32_t>(g.out_sy);
    const int64_t px = g.nx + 2 * g.h, py = g.ny + 2 * g.h, pz = g.nz + 2 * g.h;
    a.ntx = static_cast<int32_t>((px + kWaveCols - 1) / kWaveCols);
    a.nty = static_cast<int32_t>((py + RY - 1) / RY);
    a.zlen = cfg.zlen;
    a.nzc = static_cast<int32_t>((pz + cfg.zlen - 1) / cfg.zlen);
    a.wpb = cfg.wpb;
    const int64_t nblk_y = (a.nty + cfg.wpb - 1) / cfg.wpb;
    const int64_t nblocks = static_cast<int64_t>(a.ntx) * nblk_y * a.nzc;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return fail(PW_ERR_UNSUPPORTED, "grid too large");
    const dim3 grid(static_cast<unsigned>(nblocks)), block(64 * cfg.wpb);
    if constexpr (Mode != kModeGrad) {   // built for up to four wavefronts per workgroup
        if (cfg.depth == 2)
            hipLaunchKernelGGL((pw_adjoint_kernel<T, RY, 2, 256, Mode>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_adjoint_kernel<T, RY, 1, 256, Mode>), grid, block, 0, s, a);
    } else if (cfg.depth == 2) {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_adjoint_kernel<T, RY, 2, 256, Mode>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_adjoint_kernel<T, RY, 2, 512, Mode>), grid, block, 0, s, a);
    } else {
        if (cfg.wpb <= 4)
            hipLaunchKernelGGL((pw_adjoint_kernel<T, RY, 1, 256, Mode>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pw_adjoint_kernel<T, RY, 1, 512, Mode>), grid, block, 0, s, a);
    }
    return hip_fail(hipGetLastError(), "adjoint kernel launch");
}

template <typename T, int Mode>
pw_status launch_adj_dt(const AdjArgs &g, const TileCfg &cfg, double *ws, hipStream_t s) {
    switch (cfg.ry) {
        case 1: return launch_adj_t<T, 1, Mode>(g, cfg, ws, s);
        case 2: return launch_adj_t<T, 2, Mode>(g, cfg, ws, s);
        case 4: return launch_adj_t<T, 4, Mode>(g, cfg, ws, s);
        default: return fail(PW_ERR_UNSUPPORTED, "adjoint rows per strip %d not instantiated", cfg.ry);
    }
}

template <typename T>
pw_status launch_adj_mode(const AdjArgs &g, const TileCfg &cfg, int mode, double *ws, hipStream_t s) {
    TileCfg c = cfg;
    if (mode != kModeGrad && c.wpb > 4) c.wpb = 4;   // strips are independent: no result changes
    switch (mode) {
        case kModeGrad: return launch_adj_dt<T, kModeGrad>(g, c, ws, s);
        case kModeCg: return launch_adj_dt<T, kModeCg>(g, c, ws, s);
        case kModeGrad | kModeCg: return launch_adj_dt<T, kModeGrad | kModeCg>(g, c, ws, s);
    }
    return fail(PW_ERR_INVALID_ARG, "adjoint mode %d", mode);
}

}  // namespace

bool adjoint_tile_supported(const TileCfg &c) {
    return c.px == 1 && (c.depth == 1 || c.depth == 2) && (c.ry == 1 || c.ry == 2 || c.ry == 4) && c.zlen >= 1 &&
           c.wpb >= 1 && c.wpb <= 8 && c.share == 0;
}

TileCfg default_adjoint_tile(const AdjArgs &a, pw_dtype dt) {
    // Measured on MI355X (256x256x128 FP32): two-row strips, one wavefront
    // per workgroup, about 2048 wavefronts in flight.
    TileCfg c;
    c.px = 1;
    c.ry = (dt == PW_F64) ? 1 : 2;
    c.wpb = 1;
    const int64_t px = a.nx + 2 * a.h, py = a.ny + 2 * a.h, pz = a.nz + 2 * a.h;
    const int64_t strips = ((px + kWaveCols - 1) / kWaveCols) * ((py + c.ry - 1) / c.ry);
    int64_t chunks = (2048 + strips - 1) / strips;
    if (chunks < 2) chunks = 2;
    int64_t zl = (pz + chunks - 1) / chunks;
    if (zl < 8) zl = 8;
    if (zl > pz) zl = pz;
    c.zlen = static_cast<int>(zl);
    return c;
}

int64_t adjoint_strips(const pw_grid &g, int ry) {
    const int64_t px = g.nx + 2 * g.halo, py = g.ny + 2 * g.halo;
    return ((px + kWaveCols - 1) / kWaveCols) * ((py + ry - 1) / ry);
}

pw_status launch_adjoint_mode(const AdjArgs &a, pw_dtype dt, const TileCfg &cfg, bool grads, double *partials,
                              hipStream_t s) {
    if (!adjoint_tile_supported(cfg)) return fail(PW_ERR_INVALID_ARG, "unsupported adjoint tile configuration");
    const int mode = (grads ? kModeGrad : 0) | (partials ? kModeCg : 0);
    switch (dt) {
        case PW_F32: return launch_adj_mode<float>(a, cfg, mode, partials, s);
        case PW_F64: return launch_adj_mode<double>(a, cfg, mode, partials, s);
        default: return fail(PW_ERR_UNSUPPORTED, "adjoint dtype %d", static_cast<int>(dt));
    }
}

pw_status launch_adjoint(const AdjArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s) {
    return launch_adjoint_mode(a, dt, cfg, true, nullptr, s);
}

}  // namespace pw
