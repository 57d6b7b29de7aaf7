// Halo fill of padded arrays: the step before the stencil, which reads one
// layer of neighbours around the interior (Sec. 2.2).  The per-axis rules are
// documented with pw_halo_fill in pwadv.h.
//
// Every written cell lies in the halo of some axis whose rule is not KEEP,
// and its source lies in the interior of every such axis, so no cell is both
// read and written: one kernel fills all three axes with no ordering between
// its writes, and the result equals the sequential x, y, z fill.  The work of
// one field is three segments: the z-halo planes (whole rows), the y-halo
// rows of the remaining planes (whole rows) and the x-halo cells of the
// remaining rows.  A wavefront takes one piece of a whole row: its plane and
// row, their sources and value rules are found once per wavefront in scalar
// registers, and the lanes move consecutive cells, all loads before the
// stores, so that every wavefront makes one round trip to memory.  The
// x-halo cells go 64 to a wavefront in memory order (the right halo of a row
// and the left halo of the next are neighbouring lanes); in a dense array
// each row boundary still costs a cache line of its own, which only applying
// the rules by addressing (pw_advect_bc) avoids.
// Values move as raw bits (2, 4 or 8 bytes); a negated mirror flips the sign
// bit, which is exact negation.
#include <algorithm>
#include <climits>

#include "pw_internal.h"

namespace pw {
namespace {

struct HaloSeg {
    int32_t zrows, yrows;   // whole rows of the z and y segments
    int32_t xwaves;         // wavefronts of the x segment (64 cells each)
    int32_t xcells;         // cells of the x segment
    int32_t k0;             // first plane of the y and x segments
    int32_t j0, jn;         // rows covered by the x segment
    int32_t mode[3];        // x, y, z
};

struct HaloK {
    void *f[kMaxHaloFields];
    HaloSeg seg[kMaxHaloFields];
    int64_t sy, sz;
    int32_t nx, ny, nz, h;
};

// Value code of a cell, built up axis by axis in the fill's order x, y, z:
// bit 1 = the value is zero, bit 0 = the sign is flipped.  A ZERO axis sets
// the cell to +0 and drops earlier flips; a REFLECT_NEG axis after it flips
// that zero to -0, as the sequential fill does.
constexpr int kCodeNeg = 1, kCodeZero = 2;

// Source coordinate of padded coordinate p on an axis of n interior cells,
// updating the value code for a halo cell.  Padded extents fit in 32 bits.
__device__ inline int source(int p, int n, int h, int mode, int &code) {
    if (p >= h && p < n + h) return p;
    switch (mode) {
        case PW_HALO_PERIODIC: {
            int q = p - h;   // one step unless the halo is wider than the interior
            while (q < 0) q += n;
            while (q >= n) q -= n;
            return h + q;
        }
        case PW_HALO_COPY: return p < h ? h : n + h - 1;
        case PW_HALO_ZERO: code = kCodeZero; return p;
        case PW_HALO_REFLECT_NEG: code ^= kCodeNeg; [[fallthrough]];
        case PW_HALO_REFLECT: return p < h ? 2 * h - 1 - p : 2 * (n + h) - 1 - p;
        default: return p;  // KEEP
    }
}

// Composition of value codes: `first`, then `then` (see kCodeNeg).
__device__ inline int compose(int first, int then) { return (then & kCodeZero) ? then : (first ^ then); }

template <typename U> __device__ inline U coded(U x, int code) {
    const U signbit = static_cast<U>(U(1) << (8 * sizeof(U) - 1));
    const U v = (code & kCodeZero) ? U(0) : x;
    return (code & kCodeNeg) ? static_cast<U>(v ^ signbit) : v;
}

constexpr int kHaloRowCells = 4;                  // cells per lane of a row piece
constexpr int kHaloPiece = 64 * kHaloRowCells;    // cells of a row piece

// Grid: x strides over a field's wavefronts, y = field.  Wavefront w < xwaves
// takes 64 x-halo cells (first, so that their scattered round trips overlap
// the row copies), the others one piece of kHaloPiece cells of a whole row:
// one load per lane and cell, all issued before the stores.
template <typename U>
__global__ __launch_bounds__(256) void halo_kernel(HaloK a) {
    constexpr int G = kHaloRowCells;
    const int f = blockIdx.y;
    U *const base = static_cast<U *>(a.f[f]);
    const HaloSeg &s = a.seg[f];
    const int h = a.h, h2 = 2 * a.h;
    const int px = a.nx + 2 * a.h, py = a.ny + 2 * a.h;
    const int pieces = (px + kHaloPiece - 1) / kHaloPiece;
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int waves = s.xwaves + (s.zrows + s.yrows) * pieces;
    const int nwaves = static_cast<int>(gridDim.x) * 4;
    for (int wv = static_cast<int>(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
         wv < waves; wv += nwaves) {
        if (wv < s.xwaves) {   // 64 x-halo cells
            const int t = wv * 64 + lane;
            if (t < s.xcells) {
                const int r = t / h2, q = t - r * h2, c = r / s.jn;
                const int i = q < h ? q : a.nx + q;
                const int j = s.j0 + (r - c * s.jn), k = s.k0 + c;
                int code = 0;
                const int si = source(i, a.nx, h, s.mode[0], code);
                const int sj = source(j, a.ny, h, s.mode[1], code);
                const int sk = source(k, a.nz, h, s.mode[2], code);
                const U val = (code & kCodeZero) ? U(0) : base[sk * a.sz + static_cast<int64_t>(sj) * a.sy + si];
                base[k * a.sz + static_cast<int64_t>(j) * a.sy + i] = coded(val, code);
            }
        } else {               // a piece of one whole row: wave-uniform plane and row
            const int u = wv - s.xwaves, row = u / pieces, i0 = (u - row * pieces) * kHaloPiece;
            int k, j;
            if (row < s.zrows) {
                const int q = row / py;
                j = row - q * py;
                k = q < h ? q : a.nz + q;
            } else {
                const int v = row - s.zrows, c = v / h2, q = v - c * h2;
                k = s.k0 + c;
                j = q < h ? q : a.ny + q;
            }
            int cyz = 0;
            const int sj = source(j, a.ny, h, s.mode[1], cyz);
            const int sk = source(k, a.nz, h, s.mode[2], cyz);
            const U *src = base + sk * a.sz + static_cast<int64_t>(sj) * a.sy;
            U *dst = base + k * a.sz + static_cast<int64_t>(j) * a.sy;
            U val[G];
            int code[G];
#pragma unroll
            for (int m = 0; m < G; ++m) {
                const int i = i0 + 64 * m + lane;
                int cx = 0;
                const int si = source(i, a.nx, h, s.mode[0], cx);
                code[m] = cx ? compose(cx, cyz) : cyz;
                val[m] = (i < px && !(code[m] & kCodeZero)) ? src[si] : U(0);
            }
#pragma unroll
            for (int m = 0; m < G; ++m) {
                const int i = i0 + 64 * m + lane;
                if (i < px) dst[i] = coded(val[m], code[m]);
            }
        }
    }
}

// `most`: the largest number of wavefronts any field needs.
template <typename U>
hipError_t launch_u(const HaloK &k, int nf, int64_t most, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((most + 3) / 4, 16384);
    const dim3 grid(unsigned(std::max<int64_t>(blocks, 1)), unsigned(nf));
    hipLaunchKernelGGL(halo_kernel<U>, grid, dim3(256), 0, s, k);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fold
// The adjoint of the fill, one axis per launch in the order z, y, x (the
// fill is x, y, z).  A thread owns one whole line along the axis -- every
// combination of the other two padded coordinates -- and, for each halo cell
// of the line in ascending order, adds it (times the sign of the rule) into
// its source cell and clears it.  Lines are disjoint, so nothing races, and
// the order of the additions is the definition's.
struct FoldK {
    void *f[kMaxHaloFields];
    int32_t mode[kMaxHaloFields];   // rule of this axis per field
    int64_t n;                      // interior cells along the axis
    int64_t lines, inner;           // lines per field; padded extent of the faster other axis
    int64_t s_outer, s_inner, s_axis;   // strides (elements) of the slower other axis, faster other axis, the axis
    int32_t h;
};

template <typename T>
__global__ __launch_bounds__(256) void fold_kernel(FoldK a) {
    const int f = blockIdx.y;
    const int mode = a.mode[f];
    if (mode == PW_HALO_KEEP) return;   // whole workgroup
    T *const base = static_cast<T *>(a.f[f]);
    const int64_t h = a.h, n = a.n;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t l = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; l < a.lines; l += stride) {
        const int64_t o = l / a.inner, in = l - o * a.inner;
        T *const line = base + o * a.s_outer + in * a.s_inner;
        for (int64_t q = 0; q < 2 * h; ++q) {
            const int64_t p = q < h ? q : n + q;
            T *const cell = line + p * a.s_axis;
            if (mode != PW_HALO_ZERO) {
                int code = 0;
                const int64_t sp = source(static_cast<int>(p), static_cast<int>(n), static_cast<int>(h), mode, code);
                T *const dst = line + sp * a.s_axis;
                *dst = (code & kCodeNeg) ? *dst - *cell : *dst + *cell;
            }
            *cell = T(0);
        }
    }
}

}  // namespace

pw_status launch_halo_fold(const HaloArgs &a, hipStream_t s) {
    const int64_t h = a.h, px = a.nx + 2 * h, py = a.ny + 2 * h, pz = a.nz + 2 * h;
    for (int axis = 2; axis >= 0; --axis) {
        FoldK k{};
        bool any = false;
        for (int f = 0; f < a.nf; ++f) {
            k.f[f] = a.f[f];
            k.mode[f] = a.mode[f][axis];
            any = any || k.mode[f] != PW_HALO_KEEP;
        }
        if (!any) continue;
        k.h = a.h;
        if (axis == 2) {   // lines along z over (j, i)
            k.n = a.nz; k.lines = py * px; k.inner = px;
            k.s_outer = a.sy; k.s_inner = 1; k.s_axis = a.sz;
        } else if (axis == 1) {   // along y over (k, i)
            k.n = a.ny; k.lines = pz * px; k.inner = px;
            k.s_outer = a.sz; k.s_inner = 1; k.s_axis = a.sy;
        } else {   // along x over (k, j)
            k.n = a.nx; k.lines = pz * py; k.inner = py;
            k.s_outer = a.sz; k.s_inner = a.sy; k.s_axis = 1;
        }
        const int64_t blocks = std::min<int64_t>((k.lines + 255) / 256, 4096);
        const dim3 grid(unsigned(std::max<int64_t>(blocks, 1)), unsigned(a.nf));
        if (a.es == 8)
            hipLaunchKernelGGL(fold_kernel<double>, grid, dim3(256), 0, s, k);
        else
            hipLaunchKernelGGL(fold_kernel<float>, grid, dim3(256), 0, s, k);
        const pw_status st = hip_fail(hipGetLastError(), "fold kernel launch");
        if (st != PW_OK) return st;
    }
    return PW_OK;
}

pw_status launch_halo(const HaloArgs &a, hipStream_t s) {
    HaloK k{};
    k.sy = a.sy;
    k.sz = a.sz;
    k.nx = static_cast<int32_t>(a.nx);
    k.ny = static_cast<int32_t>(a.ny);
    k.nz = static_cast<int32_t>(a.nz);
    k.h = a.h;
    const int64_t h = a.h, px = a.nx + 2 * h, py = a.ny + 2 * h, pz = a.nz + 2 * h;
    int64_t most = 0;
    int nf = 0;
    for (int f = 0; f < a.nf; ++f) {
        const int32_t *m = a.mode[f];
        if (m[0] == PW_HALO_KEEP && m[1] == PW_HALO_KEEP && m[2] == PW_HALO_KEEP) continue;
        const bool fz = m[2] != PW_HALO_KEEP, fy = m[1] != PW_HALO_KEEP, fx = m[0] != PW_HALO_KEEP;
        const int64_t kn = fz ? a.nz : pz;   // planes of the y and x segments
        const int64_t jn = fy ? a.ny : py;
        const int64_t zrows = fz ? 2 * h * py : 0, yrows = fy ? kn * 2 * h : 0;
        const int64_t xcells = fx ? kn * jn * 2 * h : 0, xwaves = (xcells + 63) / 64;
        const int64_t waves = (zrows + yrows) * ((px + kHaloPiece - 1) / kHaloPiece) + xwaves;
        // 32-bit wavefront, cell and coordinate arithmetic (with room for the
        // grid-stride step)
        if (xcells + 64 > INT32_MAX || waves + 4 * 16384 > INT32_MAX || px > INT32_MAX / 2 || py > INT32_MAX / 2 ||
            pz > INT32_MAX / 2)
            return fail(PW_ERR_UNSUPPORTED, "halo fill: too many cells for 32-bit indexing");
        HaloSeg g{};
        g.zrows = static_cast<int32_t>(zrows);
        g.yrows = static_cast<int32_t>(yrows);
        g.xwaves = static_cast<int32_t>(xwaves);
        g.xcells = static_cast<int32_t>(xcells);
        g.k0 = static_cast<int32_t>(fz ? h : 0);
        g.j0 = static_cast<int32_t>(fy ? h : 0);
        g.jn = static_cast<int32_t>(jn);
        for (int d = 0; d < 3; ++d) g.mode[d] = m[d];
        k.f[nf] = a.f[f];
        k.seg[nf] = g;
        most = std::max(most, waves);
        ++nf;
    }
    if (nf == 0) return PW_OK;
    hipError_t e = hipSuccess;
    switch (a.es) {
        case 2: e = launch_u<uint16_t>(k, nf, most, s); break;
        case 4: e = launch_u<uint32_t>(k, nf, most, s); break;
        case 8: e = launch_u<uint64_t>(k, nf, most, s); break;
        default: return fail(PW_ERR_INVALID_ARG, "element size %d", a.es);
    }
    return hip_fail(e, "halo_kernel launch");
}

}  // namespace pw
