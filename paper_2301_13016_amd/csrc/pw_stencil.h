// Device-side building blocks of the forward PW stencil, shared by the
// single-grid kernel (pw_forward.hip) and the batched persistent kernel
// (pw_batch.hip).  See pw_forward.hip for the design.
#pragma once

#include "pw_internal.h"
#include "pw_lanes.h"

namespace pw {
namespace dev {

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
template <> struct Vec<float, 8> { typedef float type __attribute__((ext_vector_type(8), aligned(4))); };
template <> struct Vec<double, 2> { typedef double type __attribute__((ext_vector_type(2), aligned(8))); };
template <> struct Vec<uint16_t, 2> { typedef uint16_t type __attribute__((ext_vector_type(2), aligned(2))); };
template <> struct Vec<uint16_t, 4> { typedef uint16_t type __attribute__((ext_vector_type(4), aligned(2))); };
template <> struct Vec<_Float16, 2> { typedef _Float16 type __attribute__((ext_vector_type(2), aligned(2))); };
template <> struct Vec<_Float16, 4> { typedef _Float16 type __attribute__((ext_vector_type(4), aligned(2))); };
template <> struct Vec<uint16_t, 8> { typedef uint16_t type __attribute__((ext_vector_type(8), aligned(2))); };
template <> struct Vec<_Float16, 8> { typedef _Float16 type __attribute__((ext_vector_type(8), aligned(2))); };

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
// Cross-lane moves (pw_lanes.h): wave_shr:1 / wave_shl:1 DPP shifts, in
// which the lane with no source reads 0 and is patched from the halo.
using lanes::kWaveShl1;
using lanes::kWaveShr1;
using lanes::lane_value;
using lanes::wave_shift;

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

// Read of a kernel-invariant array at a wave-uniform index through the
// constant address space, so that it becomes a scalar load (counted apart from
// the vector loads in flight: waiting for it does not drain the prefetch).
// The caller guarantees that nothing the kernel writes overlaps the array.
template <typename T> __device__ __forceinline__ T uniform_load(const T *p, int i) {
    return ((const __attribute__((address_space(4))) T *)(p))[i];
}

// Element of type V at byte address p, read / written as global memory.  The
// kernels only touch device memory; where the array pointers come from a
// table in memory (the batched kernel) the compiler cannot infer their
// address space and would fall back to flat accesses, which wait on two
// counters.  Macros rather than templates, so that V keeps its typedef's
// (element) alignment.
#define PW_GLOAD(V, p) (*(const __attribute__((address_space(1))) V *)(p))
#define PW_GSTORE_NT(V, x, p) __builtin_nontemporal_store((x), (__attribute__((address_space(1))) V *)(p))
// Ordinary (write-back) store, for writes that cover only part of a cache
// line per instruction: L2 merges the pieces of a line before it is written
// to HBM, where separate non-temporal partial-line writes each cost HBM
// bandwidth of their own.
#define PW_GSTORE(V, x, p) (*(__attribute__((address_space(1))) V *)(p) = (x))
// Streaming read of data used once (the epilogue's addends): non-temporal, so
// it does not displace the y-halo rows that neighbouring strips re-read from L2.
#define PW_GLOAD_NT(V, p) __builtin_nontemporal_load((const __attribute__((address_space(1))) V *)(p))

using lanes::fma_;

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
    // fused epilogue (used by the Epi instantiations only): out = c + alpha * F
    const Tc *cu, *cv, *cw;
    Tc alpha;
    // boundary rules applied by addressing (pw_halo_mode per axis; KEEP reads
    // the stored halo): a read of a halo cell goes to its periodic or
    // nearest-interior source instead
    int32_t bcx = PW_HALO_KEEP, bcy = PW_HALO_KEEP, bcz = PW_HALO_KEEP;
    // value rules on top of the addressing (kernels built with Bc == 2): byte
    // d (axis x, y, z) holds a 2-bit code per field f (u, v, w) at bit 2f,
    // see bc_apply
    uint32_t bcv = 0;
};

// Padded index that a read of padded index p (0 <= p < n+2h) uses on an axis
// of n interior cells and halo h: p itself (an interior cell, or the stored
// halo under KEEP), or for a halo cell its source under the periodic or
// zero-gradient rule -- for the cells the depth-one stencil reads (p = h-1,
// p = n+h) the same map as the halo fill's, and in bounds for every p.
// Selects only, no branches: a branch between loads in flight would make the
// compiler wait for all of them where the paths join.
__device__ __forceinline__ int bc_src(int p, int n, int h, int mode) {
    const bool lo = p < h, hi = p >= n + h;
    const int per = lo ? p + n : (hi ? p - n : p);
    const int cpy = lo ? h : (hi ? n + h - 1 : p);
    return mode == PW_HALO_PERIODIC ? per : (mode == PW_HALO_COPY ? cpy : p);
}
// bc_src when the kernel is built for boundary rules (Bc), else p unchanged:
// the plain kernels carry no mapping code at all.
template <int Bc> __device__ __forceinline__ int bc_map(int p, int n, int h, int mode) {
    if constexpr (Bc) {
        return bc_src(p, n, h, mode);
    } else {
        (void)n;
        (void)h;
        (void)mode;
        return p;
    }
}

// Value rules by addressing (Bc == 2).  A halo cell's value is its source's
// value passed through one code per axis, in the halo fill's order x, y, z:
// 0 keeps it, 1 negates it (REFLECT_NEG), 2 replaces it by +0 (ZERO).  A code
// describing several axes has bit 1 = zero, bit 0 = negate: a zero drops
// what came before and a later negation turns it into -0, as the sequential
// fill does.  Codes of the three fields sit side by side, two bits each.
__device__ __forceinline__ uint32_t bc_compose(uint32_t first, uint32_t then) {   // one field
    return (then & 2u) ? then : (first ^ then);
}
__device__ __forceinline__ uint32_t bc_compose3(uint32_t first, uint32_t then) {  // three fields
    uint32_t z = then & 0x2Au;
    z |= z >> 1;   // both bits of every field whose later code zeroes
    return (then & z) | ((first ^ then) & ~z);
}
// Codes (three fields) of axis d for padded index p on an axis of n cells.
template <int Bc>
__device__ __forceinline__ uint32_t bc_axis_code(const uint32_t bcv, int d, int p, int n, int h) {
    if constexpr (Bc == 2) {
        const bool halo = p < h || p >= n + h;
        return halo ? (bcv >> (8 * d)) & 0x3Fu : 0u;
    } else {
        (void)bcv;
        (void)d;
        (void)p;
        (void)n;
        (void)h;
        return 0u;
    }
}
template <typename T> struct Bits;
template <> struct Bits<float> { using type = uint32_t; };
template <> struct Bits<double> { using type = uint64_t; };
template <> struct Bits<uint16_t> { using type = uint16_t; };
template <> struct Bits<_Float16> { using type = uint16_t; };
// x passed through code c (one field): sign-bit and zero operations on the
// stored bits, exact in every storage type.
template <typename T> __device__ __forceinline__ T bc_apply(T x, uint32_t c) {
    using B = typename Bits<T>::type;
    constexpr B sign = static_cast<B>(B(1) << (8 * sizeof(T) - 1));
    B b = __builtin_bit_cast(B, x);
    b = (c & 2u) ? B(0) : b;
    b = (c & 1u) ? static_cast<B>(b ^ sign) : b;
    return __builtin_bit_cast(T, b);
}

// One z-plane of the strip as loaded: rows 0..RY+1 are the strip's rows
// jj0-1 .. jj0+RY (interior numbering), each the lane's PX columns in storage
// precision (16-bit values stay packed two per register and are widened when
// read); hu/hv/hw are the packed halo columns (see left_of / right_of).
template <typename Tin, int PX, int RY> struct Plane {
    typename Vec<Tin, PX>::type u[RY + 2], v[RY + 2], w[RY + 2];
    Tin hu, hv, hw;
    uint32_t zcode;          // value rules: the plane's z codes (Bc == 2)
};

// Per-lane addressing of the strip, fixed for the whole march.
template <int RY> struct StripAddr {
    uint32_t roff[RY + 2];   // byte offset of this lane's first column in row r
    uint32_t hoff;           // byte offset of this lane's halo element
    int col;                 // padded column of the lane's first element
    // value rules (Bc == 2): y codes of row r (wave-uniform), the x-then-y
    // codes of this lane's halo element, and a bit per element m of the
    // lane's columns that lies in the x halo (strips at the grid's x end)
    uint32_t ycode[RY + 2];
    uint32_t yany;           // OR of ycode (wave-uniform)
    uint32_t hcode;
    uint32_t xhalo;
};

// The value rules of one freshly loaded plane, applied in place before its
// first use (Bc == 2): every row value of field f takes its x code (if its
// column is a halo column), then the row's y code, then the plane's z code.
template <typename Tin, int PX, int RY, bool Full>
__device__ __forceinline__ void bc_values(Plane<Tin, PX, RY> &P, const StripAddr<RY> &s, uint32_t bcv) {
    const uint32_t hc = bc_compose3(s.hcode, P.zcode);
    P.hu = bc_apply(P.hu, hc & 3u);
    P.hv = bc_apply(P.hv, (hc >> 2) & 3u);
    P.hw = bc_apply(P.hw, (hc >> 4) & 3u);
    // row values: only in planes or strips that reach a z or y halo, or at
    // the grid's x end (a wave-uniform test; most planes skip it)
    if (Full && (s.yany | P.zcode) == 0u) return;
    const uint32_t vx = bcv & 0x3Fu;
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const uint32_t cyz = bc_compose3(s.ycode[r], P.zcode);   // wave-uniform
#pragma unroll
        for (int m = 0; m < PX; ++m) {
            uint32_t c3 = cyz;
            if constexpr (!Full) c3 = ((s.xhalo >> m) & 1u) ? bc_compose3(vx, cyz) : cyz;
            if constexpr (PX == 1) {
                P.u[r] = bc_apply(P.u[r], c3 & 3u);
                P.v[r] = bc_apply(P.v[r], (c3 >> 2) & 3u);
                P.w[r] = bc_apply(P.w[r], (c3 >> 4) & 3u);
            } else {
                P.u[r][m] = bc_apply(P.u[r][m], c3 & 3u);
                P.v[r][m] = bc_apply(P.v[r][m], (c3 >> 2) & 3u);
                P.w[r][m] = bc_apply(P.w[r][m], (c3 >> 4) & 3u);
            }
        }
    }
}

// The value-rule codes of a strip (Bc == 2): y codes of its loaded rows
// (padded rows jj0-1+h .. jj0+RY+h, clamped as the loads are), x-then-y codes
// of the lane's packed halo element (padded row hrow_p, column hcol_p), and
// the lane's elements that lie in the x halo.
template <int Bc, int PX, int RY>
__device__ __forceinline__ void bc_strip_codes(StripAddr<RY> &s, uint32_t bcv, int jj0, int prows, int last_col,
                                               int hrow_p, int hcol_p, int nx, int ny, int h) {
    if constexpr (Bc == 2) {
        s.hcode = bc_compose3(bc_axis_code<Bc>(bcv, 0, hcol_p, nx, h), bc_axis_code<Bc>(bcv, 1, hrow_p, ny, h));
        s.xhalo = 0;
#pragma unroll
        for (int m = 0; m < PX; ++m) s.xhalo |= (min(s.col + m, last_col) >= nx + h ? 1u : 0u) << m;
        s.yany = 0;
#pragma unroll
        for (int r = 0; r < RY + 2; ++r) {
            s.ycode[r] = bc_axis_code<Bc>(bcv, 1, min(jj0 - 1 + h + r, prows - 1), ny, h);
            s.yany |= s.ycode[r];
        }
    } else {
        (void)s;
        (void)bcv;
        (void)jj0;
        (void)prows;
        (void)last_col;
        (void)hrow_p;
        (void)hcol_p;
        (void)nx;
        (void)ny;
        (void)h;
    }
}

// PX consecutive elements of one row starting at padded column `col`.  In a
// full strip (Full) every lane's vector lies inside the row and is read with
// one vector load; in the strip at the x end of the grid every lane reads
// element-wise with the columns clamped into the row (every column a stored
// output reads is in range, so clamping only affects values that are not
// used) and, in kernels built for boundary rules (Bc), then mapped by the
// axis' rule (bc_src over n interior columns, halo h).  One-column lanes need
// no clamping beyond their start column unless mapped.  The choice is made
// per wavefront, so neither path branches per lane.
template <typename Tin, int PX, bool Full, int Bc = 0>
__device__ __forceinline__ void load_row(typename Vec<Tin, PX>::type &dst, const char *plane, uint32_t off, int col,
                                         int last_col, int n, int h, int bc) {
    if constexpr (Full || (PX == 1 && !Bc)) {
        (void)col;
        (void)last_col;
        (void)n;
        (void)h;
        (void)bc;
        using VT = typename Vec<Tin, PX>::type;
        dst = PW_GLOAD(VT, plane + off);
    } else {
        const char *row = plane + off - static_cast<int64_t>(col) * static_cast<int64_t>(sizeof(Tin));
#pragma unroll
        for (int m = 0; m < PX; ++m) {
            const Tin x = PW_GLOAD(Tin, row + static_cast<int64_t>(bc_map<Bc>(min(col + m, last_col), n, h, bc)) *
                                               static_cast<int64_t>(sizeof(Tin)));
            if constexpr (PX == 1)
                dst = x;
            else
                dst[m] = x;
        }
    }
}

template <typename Tin, int PX, int RY, bool Full, int Bc = 0>
__device__ __forceinline__ void load_plane(Plane<Tin, PX, RY> &P, const FwdK<Tin> &a,
                                           int kp, const StripAddr<RY> &s, int last_col) {
    const int64_t pb = static_cast<int64_t>(kp) * a.in_sz * static_cast<int64_t>(sizeof(Tin));
    const char *bu = reinterpret_cast<const char *>(a.u) + pb;
    const char *bv = reinterpret_cast<const char *>(a.v) + pb;
    const char *bw = reinterpret_cast<const char *>(a.w) + pb;
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        load_row<Tin, PX, Full, Bc>(P.u[r], bu, s.roff[r], s.col, last_col, a.nx, a.h, a.bcx);
        load_row<Tin, PX, Full, Bc>(P.v[r], bv, s.roff[r], s.col, last_col, a.nx, a.h, a.bcx);
        load_row<Tin, PX, Full, Bc>(P.w[r], bw, s.roff[r], s.col, last_col, a.nx, a.h, a.bcx);
    }
    P.hu = PW_GLOAD(Tin, bu + s.hoff);
    P.hv = PW_GLOAD(Tin, bv + s.hoff);
    P.hw = PW_GLOAD(Tin, bw + s.hoff);
}

template <typename T, int N> __device__ __forceinline__ void store_vec(char *p, const T (&x)[N]) {
    typename Vec<T, N>::type v;
    if constexpr (N == 1) {
        v = x[0];
    } else {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = x[m];
    }
    using VT = typename Vec<T, N>::type;
    PW_GSTORE_NT(VT, v, p);
}

// The epilogue's addend rows of one output level (output layout, compute
// type): RY rows x PX columns, columns clamped into the grid (the columns
// past the end are never stored).
template <typename Tin, int PX, int RY> struct EpiRows {
    using Tc = typename Storage<Tin>::Tc;
    typename Vec<Tc, PX>::type u[RY], v[RY], w[RY];
};

template <typename Tin, int PX, int RY, bool Full>
__device__ __forceinline__ void load_epi(EpiRows<Tin, PX, RY> &E, const FwdK<Tin> &a, int kk,
                                         const uint32_t (&ooff)[RY], int ic) {
    using Tc = typename Storage<Tin>::Tc;
    const int64_t ob = static_cast<int64_t>(kk) * a.out_sz * static_cast<int64_t>(sizeof(Tc));
    const char *bu = reinterpret_cast<const char *>(a.cu) + ob;
    const char *bv = reinterpret_cast<const char *>(a.cv) + ob;
    const char *bw = reinterpret_cast<const char *>(a.cw) + ob;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        if constexpr (Full || PX == 1) {
            using VT = typename Vec<Tc, PX>::type;
            E.u[r] = PW_GLOAD_NT(VT, bu + ooff[r]);
            E.v[r] = PW_GLOAD_NT(VT, bv + ooff[r]);
            E.w[r] = PW_GLOAD_NT(VT, bw + ooff[r]);
        } else {
            // ooff is at column ic = min(ii0, nx-1); columns ic+m clamped to nx-1
#pragma unroll
            for (int m = 0; m < PX; ++m) {
                const int64_t d = static_cast<int64_t>(min(ic + m, a.nx - 1) - ic) * sizeof(Tc);
                E.u[r][m] = PW_GLOAD_NT(Tc, bu + ooff[r] + d);
                E.v[r][m] = PW_GLOAD_NT(Tc, bv + ooff[r] + d);
                E.w[r][m] = PW_GLOAD_NT(Tc, bw + ooff[r] + d);
            }
        }
    }
}

// Source terms of output level kk (interior numbering) from planes kk-1 (m),
// kk (c) and kk+1 (p); stores the lanes/rows that own outputs.
template <typename Tin, int PX, int RY, bool Full, bool Epi>
__device__ __forceinline__ void level(const Plane<Tin, PX, RY> &m, const Plane<Tin, PX, RY> &c,
                                      const Plane<Tin, PX, RY> &p,
                                      const FwdK<Tin> &a, int kk, bool lane0, bool lane63, int nvalid,
                                      const uint32_t (&ooff)[RY], const bool (&row_ok)[RY],
                                      const EpiRows<Tin, PX, RY> &E) {
    using Tc = typename Storage<Tin>::Tc;
    // element (row r, column x) of a loaded row array, widened
#define G(arr, r, x) Storage<Tin>::widen(comp<Tin, PX>((arr)[r], (x)))
#define W(h) Storage<Tin>::widen(h)
    const Tc z1 = uniform_load(a.tzc1, kk), z2 = uniform_load(a.tzc2, kk);
    const Tc d1 = uniform_load(a.tzd1, kk), d2 = uniform_load(a.tzd2, kk);
    const Tc tcx = a.tcx, tcy = a.tcy;

    // Columns just outside this lane's PX columns, per loaded row, for the
    // arrays whose x-neighbours the stencil reads.
    Tc uL[RY + 2], uR[RY + 2], vL[RY + 2], vR[RY + 2], wL[RY + 2], wR[RY + 2], wRm[RY + 2], uLp[RY + 2];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        uL[r] = left_of(G(c.u, r, PX - 1), W(c.hu), r, lane0);
        uR[r] = right_of(G(c.u, r, 0), W(c.hu), r, lane63);
        vL[r] = left_of(G(c.v, r, PX - 1), W(c.hv), r, lane0);
        vR[r] = right_of(G(c.v, r, 0), W(c.hv), r, lane63);
        wL[r] = left_of(G(c.w, r, PX - 1), W(c.hw), r, lane0);
        wR[r] = right_of(G(c.w, r, 0), W(c.hw), r, lane63);
        wRm[r] = right_of(G(m.w, r, 0), W(m.hw), r, lane63);
        uLp[r] = left_of(G(p.u, r, PX - 1), W(p.hu), r, lane0);
    }
    // value at (row r, column x-1) / (row r, column x+1) of a plane array
#define XM(arr, L, r, x) ((x) == 0 ? L[r] : G(arr, r, (x) - 1))
#define XP(arr, R, r, x) ((x) == PX - 1 ? R[r] : G(arr, r, (x) + 1))

    // Face sums shared by consecutive rows of the strip (index r = loaded row):
    //   fy = v(k,r,i) + v(k,r,i+1)   gy = v(k,r,i) + v(k,r+1,i)   hy = v(k,r,i) + v(k+1,r,i)
    Tc fy[RY + 1][PX], gy[RY + 1][PX], hy[RY + 1][PX];
#pragma unroll
    for (int r = 0; r <= RY; ++r) {
#pragma unroll
        for (int x = 0; x < PX; ++x) {
            fy[r][x] = G(c.v, r, x) + XP(c.v, vR, r, x);
            gy[r][x] = G(c.v, r, x) + G(c.v, r + 1, x);
            hy[r][x] = G(c.v, r, x) + G(p.v, r, x);
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
            const Tc uc = G(c.u, q, x);
            const Tc ul = XM(c.u, uL, q, x), ur = XP(c.u, uR, q, x);
            const Tc ax = fma_(-ur, uc + ur, ul * (uc + ul));
            const Tc ay = fma_(-G(c.u, q + 1, x), fy[q][x], G(c.u, q - 1, x) * fy[r][x]);
            const Tc fzm = G(m.w, q, x) + XP(m.w, wRm, q, x);
            const Tc fzp = G(c.w, q, x) + XP(c.w, wR, q, x);
            Tc su = tcx * ax;
            su = fma_(tcy, ay, su);
            su = fma_(z1 * G(m.u, q, x), fzm, su);
            su = fma_(-(z2 * G(p.u, q, x)), fzp, su);

            // sv: x faces (u+u at j, j+1), y faces (v+v), z faces (w+w at j, j+1)
            const Tc vl = XM(c.v, vL, q, x), vr = XP(c.v, vR, q, x);
            const Tc gxp = uc + G(c.u, q + 1, x);
            const Tc gxm = ul + XM(c.u, uL, q + 1, x);
            const Tc bx = fma_(-vr, gxp, vl * gxm);
            const Tc by = fma_(-G(c.v, q + 1, x), gy[q][x], G(c.v, q - 1, x) * gy[r][x]);
            const Tc gzm = G(m.w, q, x) + G(m.w, q + 1, x);
            const Tc gzp = G(c.w, q, x) + G(c.w, q + 1, x);
            Tc sv = tcx * bx;
            sv = fma_(tcy, by, sv);
            sv = fma_(z1 * G(m.v, q, x), gzm, sv);
            sv = fma_(-(z2 * G(p.v, q, x)), gzp, sv);

            // sw: x faces (u+u at k, k+1), y faces (v+v at k, k+1), z faces (w+w)
            const Tc wc = G(c.w, q, x);
            const Tc wl = XM(c.w, wL, q, x), wr = XP(c.w, wR, q, x);
            const Tc hxp = uc + G(p.u, q, x);
            const Tc hxm = ul + XM(p.u, uLp, q, x);
            const Tc cx = fma_(-wr, hxp, wl * hxm);
            const Tc cy = fma_(-G(c.w, q + 1, x), hy[q][x], G(c.w, q - 1, x) * hy[r][x]);
            const Tc hzm = wc + G(m.w, q, x);
            const Tc hzp = wc + G(p.w, q, x);
            Tc sw = tcx * cx;
            sw = fma_(tcy, cy, sw);
            sw = fma_(d1 * G(m.w, q, x), hzm, sw);
            sw = fma_(-(d2 * G(p.w, q, x)), hzp, sw);

            if constexpr (Epi) {   // out = c + alpha * F, one rounding
                su = fma_(a.alpha, su, comp<Tc, PX>(E.u[r], x));
                sv = fma_(a.alpha, sv, comp<Tc, PX>(E.v[r], x));
                sw = fma_(a.alpha, sw, comp<Tc, PX>(E.w[r], x));
            }
            rsu[x] = su;
            rsv[x] = sv;
            rsw[x] = sw;
        }
        if (row_ok[r]) {
            if (Full) {   // every lane owns PX columns inside the grid
                (void)nvalid;
                store_vec<Tc, PX>(osu + ooff[r], rsu);
                store_vec<Tc, PX>(osv + ooff[r], rsv);
                store_vec<Tc, PX>(osw + ooff[r], rsw);
            } else {
#pragma unroll
                for (int x = 0; x < PX; ++x) {
                    if (x < nvalid) {
                        PW_GSTORE(Tc, rsu[x], osu + ooff[r] + x * sizeof(Tc));
                        PW_GSTORE(Tc, rsv[x], osv + ooff[r] + x * sizeof(Tc));
                        PW_GSTORE(Tc, rsw[x], osw + ooff[r] + x * sizeof(Tc));
                    }
                }
            }
        }
    }
#undef XM
#undef XP
#undef G
#undef W
}

// Workgroup -> tile numbering.  Workgroups are handed to the 8 XCDs round
// robin; give XCD x the contiguous tile range [start(x), start(x+1)).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, rem) + i;
}

// One work item: the wavefront's strip (tx, ty) marched through z-chunk cz.
// All 64 lanes must be active (the cross-lane moves read every lane).  Full:
// the strip lies wholly inside the grid in x ((tx+1)*64*PX <= nx), so every
// lane loads whole vectors and owns PX outputs; otherwise loads are clamped
// element-wise (one-column lanes need no clamping beyond their start column)
// and each lane stores only its columns inside the grid.  Depth: planes in
// flight ahead of the three a level reads (1 or 2).  Epi: the fused
// epilogue out = c + alpha * F; the addend rows of level kk are loaded at the
// start of the level, before that level's plane prefetch (a scheduling
// barrier keeps the compiler from moving them after it), so waiting for them
// never waits for the prefetch.
template <typename Tin, int PX, int RY, bool Full, int Depth, bool Epi, int Bc>
__device__ __forceinline__ void strip_march_t(const FwdK<Tin> &a, int tx, int ty, int cz) {
    using Tc = typename Storage<Tin>::Tc;
    const int lane = threadIdx.x & 63;

    const int pcols = a.nx + 2 * a.h, prows = a.ny + 2 * a.h;
    const int last_col = pcols - 1;
    const int ii0 = tx * 64 * PX + lane * PX;        // first interior column of this lane
    const int nvalid = a.nx - ii0;                    // its columns inside the grid (may be <= 0)
    const int jj0 = ty * RY;

    StripAddr<RY> s;
    s.col = min(ii0 + a.h, last_col);
    // halo rows, the packed halo columns and halo planes go through the
    // boundary rules (identity under KEEP)
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int prow = bc_map<Bc>(min(jj0 - 1 + a.h + r, prows - 1), a.ny, a.h, a.bcy);
        s.roff[r] = static_cast<uint32_t>((prow * a.in_sy + s.col) * static_cast<int>(sizeof(Tin)));
    }
    {   // packed halo: lane r -> left halo of row r, lane 32+r -> right halo of row r
        const int hr = min(lane & 31, RY + 1);
        const int hrow_p = min(jj0 - 1 + a.h + hr, prows - 1);
        const int hcol_p = (lane & 32) ? min(tx * 64 * PX + 64 * PX + a.h, last_col) : tx * 64 * PX + a.h - 1;
        const int hrow = bc_map<Bc>(hrow_p, a.ny, a.h, a.bcy);
        const int hcol = bc_map<Bc>(hcol_p, a.nx, a.h, a.bcx);
        s.hoff = static_cast<uint32_t>((hrow * a.in_sy + hcol) * static_cast<int>(sizeof(Tin)));
        bc_strip_codes<Bc, PX, RY>(s, a.bcv, jj0, prows, last_col, hrow_p, hcol_p, a.nx, a.ny, a.h);
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
    const int ic = min(ii0, a.nx - 1);

    const int k0 = cz * a.zlen;
    const int k1 = min(a.nz, k0 + a.zlen);
    const int h = a.h;
    EpiRows<Tin, PX, RY> Ep;   // the epilogue's addend rows of the current level

    // The prefetch of the next plane is unconditional (near the chunk's end it
    // re-reads plane k1, a cache hit): a conditional load would merge two
    // paths with different loads in flight, and the wait inserted at such a
    // merge drains every outstanding load, prefetch included.
    // (value rules: a plane's z codes are set with its load, and the rules are
    // applied to it just before the first level that reads it)
#define PW_PLOAD(P, kp)                                                                                        \
    do {                                                                                                       \
        load_plane<Tin, PX, RY, Full, Bc>(P, a, bc_map<Bc>(min((kp), k1) + h, a.nz, h, a.bcz), s, last_col); \
        P.zcode = bc_axis_code<Bc>(a.bcv, 2, min((kp), k1) + h, a.nz, h);                                      \
    } while (0)
#define PW_LOAD(P, kp)                                                   \
    do {                                                                 \
        if constexpr (Epi) {                                             \
            load_epi<Tin, PX, RY, Full>(Ep, a, kk, ooff, ic);            \
            __builtin_amdgcn_sched_barrier(0);                           \
        }                                                                \
        PW_PLOAD(P, kp);                                                 \
    } while (0)
#define PW_LEVEL(M, C, P)                                                                      \
    do {                                                                                       \
        if constexpr (Bc == 2) bc_values<Tin, PX, RY, Full>(P, s, a.bcv);                      \
        level<Tin, PX, RY, Full, Epi>(M, C, P, a, kk, lane0, lane63, nvalid, ooff, row_ok, Ep); \
    } while (0)
#define PW_FIRST(P, kp)                                                                            \
    do {                                                                                           \
        load_plane<Tin, PX, RY, Full, Bc>(P, a, bc_map<Bc>((kp) + h, a.nz, h, a.bcz), s, last_col); \
        P.zcode = bc_axis_code<Bc>(a.bcv, 2, (kp) + h, a.nz, h);                                   \
    } while (0)
#define PW_FIX_FIRST(A, B)                                   \
    do {                                                     \
        if constexpr (Bc == 2) {                             \
            bc_values<Tin, PX, RY, Full>(A, s, a.bcv);       \
            bc_values<Tin, PX, RY, Full>(B, s, a.bcv);       \
        }                                                    \
    } while (0)
    int kk = k0;
    if constexpr (Depth == 1) {
        // four-plane ring: planes kk-1, kk, kk+1 feed level kk, kk+2 in flight
        Plane<Tin, PX, RY> A, B, C, D;
        PW_FIRST(A, k0 - 1);
        PW_PLOAD(B, k0);
        PW_PLOAD(C, k0 + 1);
        PW_FIX_FIRST(A, B);
        for (;;) {
            PW_LOAD(D, kk + 2);
            PW_LEVEL(A, B, C);
            if (++kk >= k1) break;
            PW_LOAD(A, kk + 2);
            PW_LEVEL(B, C, D);
            if (++kk >= k1) break;
            PW_LOAD(B, kk + 2);
            PW_LEVEL(C, D, A);
            if (++kk >= k1) break;
            PW_LOAD(C, kk + 2);
            PW_LEVEL(D, A, B);
            if (++kk >= k1) break;
        }
    } else {
        // five-plane ring: planes kk+2 and kk+3 in flight
        static_assert(Depth == 2, "prefetch depth 1 or 2");
        Plane<Tin, PX, RY> A, B, C, D, E;
        PW_FIRST(A, k0 - 1);
        PW_PLOAD(B, k0);
        PW_PLOAD(C, k0 + 1);
        PW_PLOAD(D, k0 + 2);
        PW_FIX_FIRST(A, B);
        for (;;) {
            PW_LOAD(E, kk + 3);
            PW_LEVEL(A, B, C);
            if (++kk >= k1) break;
            PW_LOAD(A, kk + 3);
            PW_LEVEL(B, C, D);
            if (++kk >= k1) break;
            PW_LOAD(B, kk + 3);
            PW_LEVEL(C, D, E);
            if (++kk >= k1) break;
            PW_LOAD(C, kk + 3);
            PW_LEVEL(D, E, A);
            if (++kk >= k1) break;
            PW_LOAD(D, kk + 3);
            PW_LEVEL(E, A, B);
            if (++kk >= k1) break;
        }
    }
#undef PW_PLOAD
#undef PW_LOAD
#undef PW_FIRST
#undef PW_FIX_FIRST
#undef PW_LEVEL
}

// Bc: reads go through the boundary rules a.bcx/bcy/bcz (pw_advect_bc).
template <typename Tin, int PX, int RY, int Depth, bool Epi = false, int Bc = 0>
__device__ __forceinline__ void strip_march(const FwdK<Tin> &a, int tx, int ty, int cz) {
    if constexpr (PX == 1) {
        // one-column lanes: loads never need clamping beyond the start column,
        // and one masked store per row is cheap, so one path serves every strip
        strip_march_t<Tin, PX, RY, false, Depth, Epi, Bc>(a, tx, ty, cz);
    } else if ((tx + 1) * 64 * PX <= a.nx) {
        strip_march_t<Tin, PX, RY, true, Depth, Epi, Bc>(a, tx, ty, cz);
    } else {
        strip_march_t<Tin, PX, RY, false, Depth, Epi, Bc>(a, tx, ty, cz);
    }
}

// --------------------------------------------------- strips sharing rows in LDS
// W wavefronts of one workgroup own W consecutive strips in y over the same
// columns.  Each loads only its own RY rows of every plane (plus the packed
// x-halo); the row just below and the row just above its strip are its
// neighbours' edge rows, passed through LDS, so that a row is read from
// memory once per workgroup instead of once per strip that touches it.  Only
// the workgroup's lowest wavefront reads the row below the workgroup, and its
// highest the row above.  The role of a wavefront is a template parameter, so
// the march of each role is straight-line code.
enum : int { kRoleLo = 1, kRoleMid = 2, kRoleHi = 3 };

template <typename Tin, int PX> struct LdsVec;
template <> struct LdsVec<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct LdsVec<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct LdsVec<float, 1> { typedef float type; };
template <> struct LdsVec<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct LdsVec<double, 1> { typedef double type; };
template <> struct LdsVec<uint16_t, 8> { typedef uint16_t type __attribute__((ext_vector_type(8))); };
template <> struct LdsVec<uint16_t, 4> { typedef uint16_t type __attribute__((ext_vector_type(4))); };
template <> struct LdsVec<uint16_t, 2> { typedef uint16_t type __attribute__((ext_vector_type(2))); };
template <> struct LdsVec<uint16_t, 1> { typedef uint16_t type; };
template <> struct LdsVec<_Float16, 8> { typedef _Float16 type __attribute__((ext_vector_type(8))); };
template <> struct LdsVec<_Float16, 4> { typedef _Float16 type __attribute__((ext_vector_type(4))); };
template <> struct LdsVec<_Float16, 2> { typedef _Float16 type __attribute__((ext_vector_type(2))); };
template <> struct LdsVec<_Float16, 1> { typedef _Float16 type; };

// Edge rows of one plane per slot: [slot][wavefront][0: first own row, 1:
// last own row][field][lane].  A plane's edge rows are written and read in
// the same level (before and after its barrier), and consecutive planes
// alternate between two slots.  That is enough: a wavefront writes the slot
// of plane L+1 at level L only after passing the barrier of level L-1, and
// every wavefront arrives at that barrier with all its LDS accesses
// complete (the barrier waits for them), including its reads of the same
// slot, which held plane L-1 and were made at level L-2.
constexpr int kLdsSlots = 2;
template <typename Tin, int PX, int W> struct EdgeLds {
    typename LdsVec<Tin, PX>::type e[kLdsSlots][W][2][3][64];
};

template <typename Tin, int PX>
__device__ __forceinline__ void lds_put(typename LdsVec<Tin, PX>::type &d, const typename Vec<Tin, PX>::type &x) {
    if constexpr (PX == 1) {
        d = x;
    } else {
        typename LdsVec<Tin, PX>::type t;
#pragma unroll
        for (int m = 0; m < PX; ++m) t[m] = x[m];
        d = t;
    }
}
template <typename Tin, int PX>
__device__ __forceinline__ void lds_get(typename Vec<Tin, PX>::type &d, const typename LdsVec<Tin, PX>::type &x) {
    if constexpr (PX == 1) {
        d = x;
    } else {
        const typename LdsVec<Tin, PX>::type t = x;
#pragma unroll
        for (int m = 0; m < PX; ++m) d[m] = t[m];
    }
}

// A plane's own rows (1..RY) and, by role, the row below (lowest wavefront)
// or above (highest) the workgroup, plus the packed x-halo of all RY+2 rows.
// NtOwn: rows that no other workgroup reads (not the workgroup's first or
// last own row) are read with non-temporal loads.
template <typename Tin, int PX, int RY, bool Full, int Bc, int Role, bool NtOwn = false>
__device__ __forceinline__ void load_plane_own(Plane<Tin, PX, RY> &P, const FwdK<Tin> &a, int kp,
                                               const StripAddr<RY> &s, int last_col) {
    const int64_t pb = static_cast<int64_t>(kp) * a.in_sz * static_cast<int64_t>(sizeof(Tin));
    const char *bu = reinterpret_cast<const char *>(a.u) + pb;
    const char *bv = reinterpret_cast<const char *>(a.v) + pb;
    const char *bw = reinterpret_cast<const char *>(a.w) + pb;
    constexpr int r0 = (Role == kRoleLo) ? 0 : 1;
    constexpr int r1 = (Role == kRoleHi) ? RY + 1 : RY;
#pragma unroll
    for (int r = r0; r <= r1; ++r) {
        const bool shared = r == 0 || r == RY + 1 || (Role == kRoleLo && r == 1) || (Role == kRoleHi && r == RY);
        if (NtOwn && Full && !shared) {
            using VT = typename Vec<Tin, PX>::type;
            P.u[r] = PW_GLOAD_NT(VT, bu + s.roff[r]);
            P.v[r] = PW_GLOAD_NT(VT, bv + s.roff[r]);
            P.w[r] = PW_GLOAD_NT(VT, bw + s.roff[r]);
            continue;
        }
        load_row<Tin, PX, Full, Bc>(P.u[r], bu, s.roff[r], s.col, last_col, a.nx, a.h, a.bcx);
        load_row<Tin, PX, Full, Bc>(P.v[r], bv, s.roff[r], s.col, last_col, a.nx, a.h, a.bcx);
        load_row<Tin, PX, Full, Bc>(P.w[r], bw, s.roff[r], s.col, last_col, a.nx, a.h, a.bcx);
    }
    P.hu = PW_GLOAD(Tin, bu + s.hoff);
    P.hv = PW_GLOAD(Tin, bv + s.hoff);
    P.hw = PW_GLOAD(Tin, bw + s.hoff);
}

// Publish this wavefront's edge rows of a plane: the first own row for the
// wavefront below, the last for the one above.
template <typename Tin, int PX, int RY, int W, int Role>
__device__ __forceinline__ void put_edges(EdgeLds<Tin, PX, W> &L, int slot, int wave, int lane,
                                          const Plane<Tin, PX, RY> &P) {
    if constexpr (Role != kRoleLo) {
        lds_put<Tin, PX>(L.e[slot][wave][0][0][lane], P.u[1]);
        lds_put<Tin, PX>(L.e[slot][wave][0][1][lane], P.v[1]);
        lds_put<Tin, PX>(L.e[slot][wave][0][2][lane], P.w[1]);
    }
    if constexpr (Role != kRoleHi) {
        lds_put<Tin, PX>(L.e[slot][wave][1][0][lane], P.u[RY]);
        lds_put<Tin, PX>(L.e[slot][wave][1][1][lane], P.v[RY]);
        lds_put<Tin, PX>(L.e[slot][wave][1][2][lane], P.w[RY]);
    }
}

// Take the rows just outside the strip from the neighbours' edge rows.
template <typename Tin, int PX, int RY, int W, int Role>
__device__ __forceinline__ void get_edges(const EdgeLds<Tin, PX, W> &L, int slot, int wave, int lane,
                                          Plane<Tin, PX, RY> &P) {
    if constexpr (Role != kRoleLo) {
        lds_get<Tin, PX>(P.u[0], L.e[slot][wave - 1][1][0][lane]);
        lds_get<Tin, PX>(P.v[0], L.e[slot][wave - 1][1][1][lane]);
        lds_get<Tin, PX>(P.w[0], L.e[slot][wave - 1][1][2][lane]);
    }
    if constexpr (Role != kRoleHi) {
        lds_get<Tin, PX>(P.u[RY + 1], L.e[slot][wave + 1][0][0][lane]);
        lds_get<Tin, PX>(P.v[RY + 1], L.e[slot][wave + 1][0][1][lane]);
        lds_get<Tin, PX>(P.w[RY + 1], L.e[slot][wave + 1][0][2][lane]);
    }
}

// The march of one wavefront of an LDS-sharing workgroup: as strip_march_t,
// with one barrier per level.  At level kk the wavefront publishes the edge
// rows of plane kk+1 (loaded a level earlier), waits at the barrier, and
// completes plane kk+1 with its neighbours' rows; planes kk-1 and kk were
// completed at the two levels before.  Every wavefront of the workgroup runs
// the same number of levels (same z-chunk), also one whose strip lies past
// the grid (it loads clamped rows and stores nothing), so the barriers match.
template <typename Tin, int PX, int RY, bool Full, int Depth, bool Epi, int Bc, int W, int Role, bool NtOwn = false>
__device__ __forceinline__ void strip_march_lds_t(const FwdK<Tin> &a, EdgeLds<Tin, PX, W> &L, int tx, int ty,
                                                  int cz, int wave) {
    using Tc = typename Storage<Tin>::Tc;
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
        const int prow = bc_map<Bc>(min(jj0 - 1 + a.h + r, prows - 1), a.ny, a.h, a.bcy);
        s.roff[r] = static_cast<uint32_t>((prow * a.in_sy + s.col) * static_cast<int>(sizeof(Tin)));
    }
    {
        const int hr = min(lane & 31, RY + 1);
        const int hrow_p = min(jj0 - 1 + a.h + hr, prows - 1);
        const int hcol_p = (lane & 32) ? min(tx * 64 * PX + 64 * PX + a.h, last_col) : tx * 64 * PX + a.h - 1;
        const int hrow = bc_map<Bc>(hrow_p, a.ny, a.h, a.bcy);
        const int hcol = bc_map<Bc>(hcol_p, a.nx, a.h, a.bcx);
        s.hoff = static_cast<uint32_t>((hrow * a.in_sy + hcol) * static_cast<int>(sizeof(Tin)));
        bc_strip_codes<Bc, PX, RY>(s, a.bcv, jj0, prows, last_col, hrow_p, hcol_p, a.nx, a.ny, a.h);
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
    const int ic = min(ii0, a.nx - 1);

    const int k0 = cz * a.zlen;
    const int k1 = min(a.nz, k0 + a.zlen);
    const int h = a.h;
    EpiRows<Tin, PX, RY> Ep;
    int slot = 0;   // slot of plane kk+1 at level kk: planes k0-1, k0, k0+1, ... take slots 0, 1, 2, 0, ...

    // (value rules: the raw rows go through LDS, and every wavefront applies
    // the rules to its whole plane once the neighbours' rows are in)
#define PW_PLOAD(P, kp)                                                                                            \
    do {                                                                                                           \
        load_plane_own<Tin, PX, RY, Full, Bc, Role, NtOwn>(P, a, bc_map<Bc>(min((kp), k1) + h, a.nz, h, a.bcz), s, \
                                                           last_col);                                              \
        P.zcode = bc_axis_code<Bc>(a.bcv, 2, min((kp), k1) + h, a.nz, h);                                          \
    } while (0)
#define PW_LOAD(P, kp)                                                   \
    do {                                                                 \
        if constexpr (Epi) {                                             \
            load_epi<Tin, PX, RY, Full>(Ep, a, kk, ooff, ic);            \
            __builtin_amdgcn_sched_barrier(0);                           \
        }                                                                \
        PW_PLOAD(P, kp);                                                 \
    } while (0)
#define PW_SHARE(P)                                                      \
    do {                                                                 \
        put_edges<Tin, PX, RY, W, Role>(L, slot, wave, lane, P);         \
        __syncthreads();                                                 \
        get_edges<Tin, PX, RY, W, Role>(L, slot, wave, lane, P);         \
        slot = slot == kLdsSlots - 1 ? 0 : slot + 1;                     \
        if constexpr (Bc == 2) bc_values<Tin, PX, RY, Full>(P, s, a.bcv); \
    } while (0)
#define PW_LEVEL(M, C, P)                                                                          \
    do {                                                                                           \
        PW_SHARE(P);                                                                               \
        level<Tin, PX, RY, Full, Epi>(M, C, P, a, kk, lane0, lane63, nvalid, ooff, row_ok, Ep);   \
    } while (0)
    int kk = k0;
    if constexpr (Depth == 1) {
        Plane<Tin, PX, RY> A, B, C, D;
        load_plane_own<Tin, PX, RY, Full, Bc, Role, NtOwn>(A, a, bc_map<Bc>(k0 - 1 + h, a.nz, h, a.bcz), s, last_col);
        A.zcode = bc_axis_code<Bc>(a.bcv, 2, k0 - 1 + h, a.nz, h);
        PW_PLOAD(B, k0);
        PW_PLOAD(C, k0 + 1);
        PW_SHARE(A);
        PW_SHARE(B);
        for (;;) {
            PW_LOAD(D, kk + 2);
            PW_LEVEL(A, B, C);
            if (++kk >= k1) break;
            PW_LOAD(A, kk + 2);
            PW_LEVEL(B, C, D);
            if (++kk >= k1) break;
            PW_LOAD(B, kk + 2);
            PW_LEVEL(C, D, A);
            if (++kk >= k1) break;
            PW_LOAD(C, kk + 2);
            PW_LEVEL(D, A, B);
            if (++kk >= k1) break;
        }
    } else {
        static_assert(Depth == 2, "prefetch depth 1 or 2");
        Plane<Tin, PX, RY> A, B, C, D, E;
        load_plane_own<Tin, PX, RY, Full, Bc, Role, NtOwn>(A, a, bc_map<Bc>(k0 - 1 + h, a.nz, h, a.bcz), s, last_col);
        A.zcode = bc_axis_code<Bc>(a.bcv, 2, k0 - 1 + h, a.nz, h);
        PW_PLOAD(B, k0);
        PW_PLOAD(C, k0 + 1);
        PW_PLOAD(D, k0 + 2);
        PW_SHARE(A);
        PW_SHARE(B);
        for (;;) {
            PW_LOAD(E, kk + 3);
            PW_LEVEL(A, B, C);
            if (++kk >= k1) break;
            PW_LOAD(A, kk + 3);
            PW_LEVEL(B, C, D);
            if (++kk >= k1) break;
            PW_LOAD(B, kk + 3);
            PW_LEVEL(C, D, E);
            if (++kk >= k1) break;
            PW_LOAD(C, kk + 3);
            PW_LEVEL(D, E, A);
            if (++kk >= k1) break;
            PW_LOAD(D, kk + 3);
            PW_LEVEL(E, A, B);
            if (++kk >= k1) break;
        }
    }
#undef PW_PLOAD
#undef PW_LOAD
#undef PW_SHARE
#undef PW_LEVEL
}

// Dispatch of one wavefront of an LDS-sharing workgroup to its role's march
// (the wave index is wave-uniform, so this branch is taken once, before any
// load), and to the full-strip or x-edge path.
template <typename Tin, int PX, int RY, int Depth, bool Epi, int Bc, int W, bool Full, bool NtOwn>
__device__ __forceinline__ void strip_march_lds_f(const FwdK<Tin> &a, EdgeLds<Tin, PX, W> &L, int tx, int ty,
                                                  int cz, int wave) {
    static_assert(W >= 2, "sharing needs two wavefronts or more");
    if (wave == 0)
        strip_march_lds_t<Tin, PX, RY, Full, Depth, Epi, Bc, W, kRoleLo, NtOwn>(a, L, tx, ty, cz, wave);
    else if (wave == W - 1)
        strip_march_lds_t<Tin, PX, RY, Full, Depth, Epi, Bc, W, kRoleHi, NtOwn>(a, L, tx, ty, cz, wave);
    else if constexpr (W > 2)
        strip_march_lds_t<Tin, PX, RY, Full, Depth, Epi, Bc, W, kRoleMid, NtOwn>(a, L, tx, ty, cz, wave);
}

template <typename Tin, int PX, int RY, int Depth, bool Epi, int Bc, int W, bool NtOwn = false>
__device__ __forceinline__ void strip_march_lds(const FwdK<Tin> &a, EdgeLds<Tin, PX, W> &L, int tx, int ty, int cz,
                                                int wave) {
    if constexpr (PX == 1) {
        strip_march_lds_f<Tin, PX, RY, Depth, Epi, Bc, W, false, NtOwn>(a, L, tx, ty, cz, wave);
    } else if ((tx + 1) * 64 * PX <= a.nx) {
        strip_march_lds_f<Tin, PX, RY, Depth, Epi, Bc, W, true, NtOwn>(a, L, tx, ty, cz, wave);
    } else {
        strip_march_lds_f<Tin, PX, RY, Depth, Epi, Bc, W, false, NtOwn>(a, L, tx, ty, cz, wave);
    }
}

}  // namespace dev
}  // namespace pw
