// Gradients of L = <su, gsu> + <sv, gsv> + <sw, gsw> with respect to the
// coefficients, gfx950.  L is linear in every coefficient: each term of the
// operator is one coefficient times a coefficient-free product, so dL/dc sums,
// over the terms c multiplies, the cotangent at the term's output point times
// that product.  tcx and tcy multiply the x- and y-face terms at every point;
// tzc1[k], tzc2[k] (u, v) and tzd1[k], tzd2[k] (w) the lower / upper z-face
// terms of level k.
//
// Pass 1 (the strip march of the forward kernel, fixed launch shape): every
// wavefront evaluates the six coefficient-free term groups at its points,
// weights them by the cotangents, sums per lane in FP64 and then across the
// wavefront, and writes one partial per (quantity, level, strip) to the
// workspace.  Pass 2 sums the strips of each (quantity, level) in a fixed
// order, and pass 3 the levels of tcx and tcy.  No atomics: the result is the
// same on every run.
#include <mutex>

#include "pw_stencil.h"

namespace pw {
namespace {

using namespace dev;

constexpr int kQ = 6;   // tzc1, tzc2, tzd1, tzd2, tcx (level share), tcy (level share)

template <typename T> struct CgK {
    FwdK<T> x;                    // values and shape (the coefficient and output fields are unused)
    const T *ru, *rv, *rw;        // cotangents, output layout
    double *ws;                   // [kQ][nz][nstrips]
    int32_t nstrips;
};

// Fixed launch shape: strips of 64*PX columns x RY rows.
template <typename T> struct CgShape;
template <> struct CgShape<float> {
    static constexpr int PX = 2, RY = 2;
};
template <> struct CgShape<double> {
    static constexpr int PX = 1, RY = 2;
};

// x moved across lanes by a DPP control that gives every lane a source (a
// permutation within quads or rows), both halves of the double.
template <int Ctrl> __device__ __forceinline__ double dpp_move(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), Ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), Ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowRor4 = 0x124;   // rotate by 4 within a row of 16 lanes
constexpr int kRowRor8 = 0x128;   // rotate by 8

// Sum over the 64 lanes, the same value in every lane and the same order on
// every run: pairs and quads (quad permutations), the four quads of each
// 16-lane row (row rotations), then the four row sums in a fixed order.  All
// register moves (DPP, readlane): no LDS traffic and no waits.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_move<kQuadXor1>(x);
    x += dpp_move<kQuadXor2>(x);
    x += dpp_move<kRowRor4>(x);
    x += dpp_move<kRowRor8>(x);
    return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}

// Cotangent rows of one output level: RY rows x PX columns, clamped (rows and
// columns outside the grid are masked by the caller).
template <typename T, int PX, int RY> struct CotRows {
    typename Vec<T, PX>::type u[RY], v[RY], w[RY];
};

template <typename T, int PX, int RY, bool Full>
__device__ __forceinline__ void load_cot(CotRows<T, PX, RY> &R, const CgK<T> &g, int kk, const uint32_t (&ooff)[RY],
                                         int ic, int nx) {
    const int64_t ob = static_cast<int64_t>(kk) * g.x.out_sz * static_cast<int64_t>(sizeof(T));
    const char *bu = reinterpret_cast<const char *>(g.ru) + ob;
    const char *bv = reinterpret_cast<const char *>(g.rv) + ob;
    const char *bw = reinterpret_cast<const char *>(g.rw) + ob;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        if constexpr (Full || PX == 1) {
            using VT = typename Vec<T, PX>::type;
            R.u[r] = PW_GLOAD(VT, bu + ooff[r]);
            R.v[r] = PW_GLOAD(VT, bv + ooff[r]);
            R.w[r] = PW_GLOAD(VT, bw + ooff[r]);
        } else {
            // ooff points at column ic = min(ii0, nx-1); read columns ii0+m clamped
#pragma unroll
            for (int m = 0; m < PX; ++m) {
                const int64_t d = static_cast<int64_t>(min(ic + m, nx - 1) - ic) * sizeof(T);
                R.u[r][m] = PW_GLOAD(T, bu + ooff[r] + d);
                R.v[r][m] = PW_GLOAD(T, bv + ooff[r] + d);
                R.w[r][m] = PW_GLOAD(T, bw + ooff[r] + d);
            }
        }
    }
}

// The six cotangent-weighted term groups of level kk, summed over the lane's
// PX x RY points in the compute type (a handful of terms: at most three
// roundings of 2^-24 relative to the sum of magnitudes in FP32) and handed
// over in FP64, in which the wavefront and the strips are summed.
template <typename T, int PX, int RY, bool Full>
__device__ __forceinline__ void level_cg(const Plane<T, PX, RY> &m, const Plane<T, PX, RY> &c,
                                         const Plane<T, PX, RY> &p, const CotRows<T, PX, RY> &R, bool lane0,
                                         bool lane63, int nvalid, const bool (&row_ok)[RY], double (&acc)[kQ]) {
#define G(arr, r, x) comp<T, PX>((arr)[r], (x))
    T uL[RY + 2], uR[RY + 2], vR[RY + 2], vL[RY + 2], wL[RY + 2], wR[RY + 2], wRm[RY + 2], uLp[RY + 2];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        uL[r] = left_of(G(c.u, r, PX - 1), c.hu, r, lane0);
        uR[r] = right_of(G(c.u, r, 0), c.hu, r, lane63);
        vL[r] = left_of(G(c.v, r, PX - 1), c.hv, r, lane0);
        vR[r] = right_of(G(c.v, r, 0), c.hv, r, lane63);
        wL[r] = left_of(G(c.w, r, PX - 1), c.hw, r, lane0);
        wR[r] = right_of(G(c.w, r, 0), c.hw, r, lane63);
        wRm[r] = right_of(G(m.w, r, 0), m.hw, r, lane63);
        uLp[r] = left_of(G(p.u, r, PX - 1), p.hu, r, lane0);
    }
#define XM(arr, L, r, x) ((x) == 0 ? L[r] : G(arr, r, (x) - 1))
#define XP(arr, Rr, r, x) ((x) == PX - 1 ? Rr[r] : G(arr, r, (x) + 1))
    T s[kQ] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int q = r + 1;
#pragma unroll
        for (int x = 0; x < PX; ++x) {
            const bool ok = row_ok[r] && (Full || x < nvalid);
            const T a = ok ? comp<T, PX>(R.u[r], x) : T(0);
            const T b = ok ? comp<T, PX>(R.v[r], x) : T(0);
            const T e = ok ? comp<T, PX>(R.w[r], x) : T(0);
            // su term groups
            const T uc = G(c.u, q, x), ul = XM(c.u, uL, q, x), ur = XP(c.u, uR, q, x);
            const T ax = fma_(-ur, uc + ur, ul * (uc + ul));
            const T fy0 = G(c.v, q - 1, x) + XP(c.v, vR, q - 1, x), fy1 = G(c.v, q, x) + XP(c.v, vR, q, x);
            const T ay = fma_(-G(c.u, q + 1, x), fy1, G(c.u, q - 1, x) * fy0);
            const T az1 = G(m.u, q, x) * (G(m.w, q, x) + XP(m.w, wRm, q, x));
            const T az2 = G(p.u, q, x) * (G(c.w, q, x) + XP(c.w, wR, q, x));
            // sv term groups
            const T vc = G(c.v, q, x), vl = XM(c.v, vL, q, x), vr = XP(c.v, vR, q, x);
            const T bx = fma_(-vr, uc + G(c.u, q + 1, x), vl * (ul + XM(c.u, uL, q + 1, x)));
            const T by = fma_(-G(c.v, q + 1, x), vc + G(c.v, q + 1, x), G(c.v, q - 1, x) * (vc + G(c.v, q - 1, x)));
            const T bz1 = G(m.v, q, x) * (G(m.w, q, x) + G(m.w, q + 1, x));
            const T bz2 = G(p.v, q, x) * (G(c.w, q, x) + G(c.w, q + 1, x));
            // sw term groups
            const T wc = G(c.w, q, x), wl = XM(c.w, wL, q, x), wr = XP(c.w, wR, q, x);
            const T cx = fma_(-wr, uc + G(p.u, q, x), wl * (ul + XM(p.u, uLp, q, x)));
            const T cy = fma_(-G(c.w, q + 1, x), G(c.v, q, x) + G(p.v, q, x),
                              G(c.w, q - 1, x) * (G(c.v, q - 1, x) + G(p.v, q - 1, x)));
            const T cz1 = G(m.w, q, x) * (wc + G(m.w, q, x));
            const T cz2 = G(p.w, q, x) * (wc + G(p.w, q, x));
            // A point outside the interior reads clamped cells, which may
            // hold anything (a NaN there times a zero cotangent is NaN), so
            // its contributions are selected away, not multiplied away.
            s[0] += ok ? fma_(a, az1, b * bz1) : T(0);
            s[1] -= ok ? fma_(a, az2, b * bz2) : T(0);
            s[2] += ok ? e * cz1 : T(0);
            s[3] -= ok ? e * cz2 : T(0);
            s[4] += ok ? fma_(a, ax, fma_(b, bx, e * cx)) : T(0);
            s[5] += ok ? fma_(a, ay, fma_(b, by, e * cy)) : T(0);
        }
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) acc[q] = static_cast<double>(s[q]);
#undef G
#undef XM
#undef XP
}

template <typename T, int PX, int RY, bool Full>
__device__ __forceinline__ void cg_march(const CgK<T> &g, int tx, int ty, int cz) {
    const FwdK<T> &a = g.x;
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
    const int ic = min(ii0, a.nx - 1);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row_ok[r] = jj0 + r < a.ny;
        const int jj = min(jj0 + r, a.ny - 1);
        ooff[r] = static_cast<uint32_t>((jj * a.out_sy + ic) * static_cast<int>(sizeof(T)));
    }
    const bool lane0 = lane == 0, lane63 = lane == 63;
    const int k0 = cz * a.zlen;
    const int k1 = min(a.nz, k0 + a.zlen);
    const int h = a.h;
    const int strip = ty * a.ntx + tx;

    // As the forward march: a four-plane ring of values with plane kk+2 in
    // flight, and the cotangents of level kk+1 loaded during level kk; every
    // load unconditional (clamped), so no wait drains the prefetch.
    Plane<T, PX, RY> A, B, C, D;
    CotRows<T, PX, RY> R0, R1;
    load_plane<T, PX, RY, Full>(A, a, k0 - 1 + h, s, last_col);
    load_plane<T, PX, RY, Full>(B, a, k0 + h, s, last_col);
    load_plane<T, PX, RY, Full>(C, a, k0 + 1 + h, s, last_col);
    load_cot<T, PX, RY, Full>(R0, g, k0, ooff, ic, a.nx);
    auto emit = [&](int kk, const double (&acc)[kQ]) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const double t = wave_sum(acc[q]);
            if (lane0) g.ws[(static_cast<int64_t>(q) * a.nz + kk) * g.nstrips + strip] = t;
        }
    };
#define PW_CG_LEVEL(M, Cc, P, RC, RN)                                                   \
    do {                                                                                \
        load_cot<T, PX, RY, Full>(RN, g, min(kk + 1, k1 - 1), ooff, ic, a.nx);          \
        double acc[kQ] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};                                \
        level_cg<T, PX, RY, Full>(M, Cc, P, RC, lane0, lane63, nvalid, row_ok, acc);    \
        emit(kk, acc);                                                                  \
    } while (0)
    int kk = k0;
    for (;;) {
        load_plane<T, PX, RY, Full>(D, a, min(kk + 2, k1) + h, s, last_col);
        PW_CG_LEVEL(A, B, C, R0, R1);
        if (++kk >= k1) break;
        load_plane<T, PX, RY, Full>(A, a, min(kk + 2, k1) + h, s, last_col);
        PW_CG_LEVEL(B, C, D, R1, R0);
        if (++kk >= k1) break;
        load_plane<T, PX, RY, Full>(B, a, min(kk + 2, k1) + h, s, last_col);
        PW_CG_LEVEL(C, D, A, R0, R1);
        if (++kk >= k1) break;
        load_plane<T, PX, RY, Full>(C, a, min(kk + 2, k1) + h, s, last_col);
        PW_CG_LEVEL(D, A, B, R1, R0);
        if (++kk >= k1) break;
    }
#undef PW_CG_LEVEL
}

template <typename T>
__global__ __launch_bounds__(256) void pw_coeffgrad_kernel(CgK<T> g) {
    constexpr int PX = CgShape<T>::PX, RY = CgShape<T>::RY;
    const FwdK<T> &a = g.x;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int cz = t % a.nzc;
    const int t2 = t / a.nzc;
    const int tx = t2 % a.ntx;
    const int ty = (t2 / a.ntx) * a.wpb + wave;
    if (ty >= a.nty) return;   // whole wavefront
    if constexpr (PX == 1) {
        cg_march<T, PX, RY, false>(g, tx, ty, cz);
    } else if ((tx + 1) * 64 * PX <= a.nx) {
        cg_march<T, PX, RY, true>(g, tx, ty, cz);
    } else {
        cg_march<T, PX, RY, false>(g, tx, ty, cz);
    }
}

// Pass 2: out[q*nz + k] = sum over strips of ws[q][k][strip], one workgroup
// per (q, k), a fixed order (strided per thread, then a tree in LDS).
__global__ __launch_bounds__(256) void pw_coeffgrad_reduce_kernel(const double *__restrict__ ws, int64_t nstrips,
                                                                  double *__restrict__ out) {
    __shared__ double part[256];
    const double *row = ws + static_cast<int64_t>(blockIdx.x) * nstrips;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nstrips; i += 256) s += row[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// Pass 3: out[6*nz + q] = sum over levels of the tcx (q = 0) / tcy (q = 1)
// level shares; wavefront q adds lane-strided levels, then a butterfly (a
// fixed order).
__global__ __launch_bounds__(128) void pw_coeffgrad_total_kernel(double *__restrict__ out, int nz) {
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double *lv = out + (4 + q) * nz;
    double s = 0.0;
    for (int k = lane; k < nz; k += 64) s += lv[k];
    s = wave_sum(s);
    if (lane == 0) out[6 * nz + q] = s;
}

template <typename T> CgK<T> make_args(const CgArgs &g, int64_t *nstrips_out, int64_t *nblocks_out) {
    constexpr int PX = CgShape<T>::PX, RY = CgShape<T>::RY;
    CgK<T> k;
    FwdK<T> &a = k.x;
    a.u = static_cast<const T *>(g.u);
    a.v = static_cast<const T *>(g.v);
    a.w = static_cast<const T *>(g.w);
    a.su = a.sv = a.sw = nullptr;
    a.tzc1 = a.tzc2 = a.tzd1 = a.tzd2 = nullptr;
    a.tcx = a.tcy = T(0);
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
    a.wpb = 1;
    const int64_t nstrips = static_cast<int64_t>(a.ntx) * a.nty;
    // about 2048 wavefronts: cut the march into z-chunks when there are few strips
    int64_t chunks = (2048 + nstrips - 1) / nstrips;
    if (chunks < 1) chunks = 1;
    int64_t zl = (g.nz + chunks - 1) / chunks;
    if (zl < 8) zl = 8;
    if (zl > g.nz) zl = g.nz;
    a.zlen = static_cast<int32_t>(zl);
    a.nzc = static_cast<int32_t>((g.nz + zl - 1) / zl);
    k.ru = static_cast<const T *>(g.gsu);
    k.rv = static_cast<const T *>(g.gsv);
    k.rw = static_cast<const T *>(g.gsw);
    k.ws = static_cast<double *>(g.workspace);
    k.nstrips = static_cast<int32_t>(nstrips);
    *nstrips_out = nstrips;
    *nblocks_out = nstrips * a.nzc;
    return k;
}

template <typename T> pw_status launch_cg_t(const CgArgs &g, hipStream_t s) {
    int64_t nstrips = 0, nblocks = 0;
    const CgK<T> k = make_args<T>(g, &nstrips, &nblocks);
    if (nblocks <= 0 || nblocks > 0x7fffffffLL || nstrips > 0x7fffffffLL)
        return fail(PW_ERR_UNSUPPORTED, "grid too large");
    hipLaunchKernelGGL(pw_coeffgrad_kernel<T>, dim3(static_cast<unsigned>(nblocks)), dim3(64), 0, s, k);
    pw_status st = hip_fail(hipGetLastError(), "coefficient gradient kernel launch");
    if (st != PW_OK) return st;
    hipLaunchKernelGGL(pw_coeffgrad_reduce_kernel, dim3(static_cast<unsigned>(kQ * g.nz)), dim3(256), 0, s,
                       static_cast<const double *>(g.workspace), nstrips, static_cast<double *>(g.grad));
    st = hip_fail(hipGetLastError(), "coefficient gradient reduction launch");
    if (st != PW_OK) return st;
    hipLaunchKernelGGL(pw_coeffgrad_total_kernel, dim3(1), dim3(128), 0, s, static_cast<double *>(g.grad),
                       static_cast<int>(g.nz));
    return hip_fail(hipGetLastError(), "coefficient gradient total launch");
}

// Scratch of the allocation-free entry point (pw_advect_coeff_grad_static):
// the per-strip partials of one call live in this array instead of a caller
// workspace.  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never uses the array's name as an address (on the
// host it is a stand-in, not device memory); it uses the address that
// hipGetSymbolAddress returns on each device.
static __device__ __align__(256) double scratch[kCoeffGradScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

}  // namespace

pw_status coeff_grad_scratch(void **ptr) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PW_ERR_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e2 = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e2 != hipSuccess) return hip_fail(e2, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PW_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PW_OK;
}

int64_t coeff_grad_workspace_bytes(const pw_grid &g, pw_dtype dt) {
    const int px = dt == PW_F64 ? CgShape<double>::PX : CgShape<float>::PX;
    const int ry = dt == PW_F64 ? CgShape<double>::RY : CgShape<float>::RY;
    const int64_t nstrips = ((g.nx + 64 * px - 1) / (64 * px)) * ((g.ny + ry - 1) / ry);
    return kQ * g.nz * nstrips * static_cast<int64_t>(sizeof(double));
}

pw_status launch_coeff_grad(const CgArgs &a, pw_dtype dt, hipStream_t s) {
    switch (dt) {
        case PW_F32: return launch_cg_t<float>(a, s);
        case PW_F64: return launch_cg_t<double>(a, s);
        default: return fail(PW_ERR_UNSUPPORTED, "coefficient gradients support PW_F32 and PW_F64 only");
    }
}

}  // namespace pw
