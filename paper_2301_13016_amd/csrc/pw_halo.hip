// Halo fill of padded arrays: the step before the stencil, which reads one
// layer of neighbours around the interior (Sec. 2.2).  The per-axis rules are
// documented with pw_halo_fill in pwadv.h.
//
// Every written cell lies in the halo of some axis whose rule is not KEEP,
// and its source lies in the interior of every such axis, so no cell is both
// read and written: one kernel fills all three axes with no ordering between
// its writes, and the result equals the sequential x, y, z fill.  The work of
// one field is three segments: the z-halo planes (whole planes), the y-halo
// rows of the remaining planes (whole rows) and the x-halo cells of the
// remaining rows.  The first two are whole rows: one wavefront takes a row,
// finds its source row once, and its lanes move consecutive cells (coalesced
// loads and stores, per-cell work only on the x axis).  The x-halo cells are
// scattered, one per thread.  Values move as raw bits (2, 4 or 8 bytes); a
// negated mirror flips the sign bit, which is exact negation.
#include <algorithm>

#include "pw_internal.h"

namespace pw {
namespace {

struct HaloSeg {
    int64_t nzs, nys, nxs;  // rows of the z and y segments, cells of the x segment
    int64_t k0, kn;         // planes covered by the y and x segments
    int64_t j0, jn;         // rows covered by the x segment
    int32_t mode[3];        // x, y, z
};

struct HaloK {
    void *f[kMaxHaloFields];
    HaloSeg seg[kMaxHaloFields];
    int64_t nx, ny, nz, sy, sz;
    int32_t h;
};

// Source coordinate of padded coordinate p on an axis of n interior cells;
// `sign` becomes 0 for a zeroed cell and flips for a negated mirror.
__device__ inline int64_t source(int64_t p, int64_t n, int64_t h, int mode, int &sign) {
    if (p >= h && p < n + h) return p;
    switch (mode) {
        case PW_HALO_PERIODIC: {
            int64_t q = (p - h) % n;
            return h + (q < 0 ? q + n : q);
        }
        case PW_HALO_COPY: return p < h ? h : n + h - 1;
        case PW_HALO_ZERO: sign = 0; return p;
        case PW_HALO_REFLECT_NEG: sign = -sign; [[fallthrough]];
        case PW_HALO_REFLECT: return p < h ? 2 * h - 1 - p : 2 * (n + h) - 1 - p;
        default: return p;  // KEEP
    }
}

// I: index type of the work decomposition (32-bit when every count fits, to
// keep the divisions cheap).  Grid: x strides over a field's work, y = field.
template <typename U, typename I>
__global__ __launch_bounds__(256) void halo_kernel(HaloK a) {
    const int f = blockIdx.y;
    U *const base = static_cast<U *>(a.f[f]);
    const HaloSeg &s = a.seg[f];
    const I h = I(a.h), h2 = I(2 * a.h);
    const I px = I(a.nx + 2 * a.h), py = I(a.ny + 2 * a.h);
    const U signbit = U(1) << (8 * sizeof(U) - 1);

    // whole rows: the z-halo planes (row index r < nzs) and the y-halo rows of
    // the other planes; one wavefront per row
    const I rows = I(s.nzs + s.nys), nzs = I(s.nzs);
    const int lane = static_cast<int>(threadIdx.x & 63);
    const I nwaves = I(gridDim.x) * I(blockDim.x >> 6);
    const I wave0 = I(blockIdx.x) * I(blockDim.x >> 6) + I(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    for (I r = wave0; r < rows; r += nwaves) {
        int64_t k, j;
        if (r < nzs) {
            const I q = r / py;
            j = r - q * py;
            k = q < h ? q : a.nz + q;
        } else {
            const I u = r - nzs, c = u / h2, q = u - c * h2;
            k = s.k0 + c;
            j = q < h ? q : a.ny + q;
        }
        int sign_kj = 1;
        const int64_t sj = source(j, a.ny, a.h, s.mode[1], sign_kj);
        const int64_t sk = source(k, a.nz, a.h, s.mode[2], sign_kj);
        const U *src = base + sk * a.sz + sj * a.sy;
        U *dst = base + k * a.sz + j * a.sy;
        for (int64_t i = lane; i < int64_t(px); i += 64) {
            int sign = sign_kj;
            const int64_t si = source(i, a.nx, a.h, s.mode[0], sign);
            U val = 0;
            if (sign != 0) {
                val = src[si];
                if (sign < 0) val ^= signbit;
            }
            dst[i] = val;
        }
    }

    // the x-halo cells of the remaining rows, one per thread
    const I cells = I(s.nxs), jn = I(s.jn);
    const I stride = I(gridDim.x) * I(blockDim.x);
    for (I t = I(blockIdx.x) * I(blockDim.x) + I(threadIdx.x); t < cells; t += stride) {
        const I r = t / h2, c = r / jn, q = t - r * h2;
        const int64_t j = s.j0 + (r - c * jn);
        const int64_t k = s.k0 + c;
        const int64_t i = q < h ? q : a.nx + q;
        int sign = 1;
        const int64_t si = source(i, a.nx, a.h, s.mode[0], sign);
        const int64_t sj = source(j, a.ny, a.h, s.mode[1], sign);
        const int64_t sk = source(k, a.nz, a.h, s.mode[2], sign);
        U val = 0;
        if (sign != 0) {
            val = base[sk * a.sz + sj * a.sy + si];
            if (sign < 0) val ^= signbit;
        }
        base[k * a.sz + j * a.sy + i] = val;
    }
}

// `most`: the largest number of blocks any field's work asks for.
template <typename U>
hipError_t launch_u(const HaloK &k, int nf, int64_t most, bool small, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>(most, 2048);
    const dim3 grid(unsigned(std::max<int64_t>(blocks, 1)), unsigned(nf));
    if (small)
        hipLaunchKernelGGL((halo_kernel<U, uint32_t>), grid, dim3(256), 0, s, k);
    else
        hipLaunchKernelGGL((halo_kernel<U, uint64_t>), grid, dim3(256), 0, s, k);
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
                int sign = 1;
                const int64_t sp = source(p, n, h, mode, sign);
                T *const dst = line + sp * a.s_axis;
                *dst = sign < 0 ? *dst - *cell : *dst + *cell;
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
    k.nx = a.nx;
    k.ny = a.ny;
    k.nz = a.nz;
    k.sy = a.sy;
    k.sz = a.sz;
    k.h = a.h;
    const int64_t h = a.h, px = a.nx + 2 * h, py = a.ny + 2 * h, pz = a.nz + 2 * h;
    int64_t most = 0;
    int nf = 0;
    for (int f = 0; f < a.nf; ++f) {
        const int32_t *m = a.mode[f];
        if (m[0] == PW_HALO_KEEP && m[1] == PW_HALO_KEEP && m[2] == PW_HALO_KEEP) continue;
        HaloSeg g{};
        const bool fz = m[2] != PW_HALO_KEEP, fy = m[1] != PW_HALO_KEEP, fx = m[0] != PW_HALO_KEEP;
        g.k0 = fz ? h : 0;
        g.kn = fz ? a.nz : pz;
        g.j0 = fy ? h : 0;
        g.jn = fy ? a.ny : py;
        g.nzs = fz ? 2 * h * py : 0;        // rows
        g.nys = fy ? g.kn * 2 * h : 0;      // rows
        g.nxs = fx ? g.kn * g.jn * 2 * h : 0;   // cells
        for (int d = 0; d < 3; ++d) g.mode[d] = m[d];
        k.f[nf] = a.f[f];
        k.seg[nf] = g;
        // four rows per block (one per wavefront), 256 cells per block
        most = std::max({most, (g.nzs + g.nys + 3) / 4, (g.nxs + 255) / 256});
        ++nf;
    }
    if (nf == 0) return PW_OK;
    // 32-bit decomposition when every count and a loop's last increment fit
    int64_t biggest = 0;
    for (int f = 0; f < nf; ++f) biggest = std::max({biggest, k.seg[f].nzs + k.seg[f].nys, k.seg[f].nxs});
    const bool small = biggest + 2048 * 256 < (int64_t(1) << 32) && px * py < (int64_t(1) << 32);
    hipError_t e = hipSuccess;
    switch (a.es) {
        case 2: e = launch_u<uint16_t>(k, nf, most, small, s); break;
        case 4: e = launch_u<uint32_t>(k, nf, most, small, s); break;
        case 8: e = launch_u<uint64_t>(k, nf, most, small, s); break;
        default: return fail(PW_ERR_INVALID_ARG, "element size %d", a.es);
    }
    return hip_fail(e, "halo_kernel launch");
}

}  // namespace pw
