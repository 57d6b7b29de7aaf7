// C ABI of libpwadv: argument validation, error reporting and dispatch to the
// kernel launchers.  Declarations and the contract are in include/pwadv.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "pw_internal.h"

namespace pw {

static thread_local char g_err[512] = "";

pw_status fail(pw_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

pw_status hip_fail(hipError_t e, const char *what) {
    if (e == hipSuccess) return PW_OK;
    return fail(PW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// PWADV_LOG (set and not "0"): one line on stderr per launch -- entry point,
// grid, storage type, launch shape and where the shape came from.  Read once
// per process.
static bool log_enabled() {
    static const bool on = [] {
        const char *e = std::getenv("PWADV_LOG");
        return e != nullptr && e[0] != '\0' && std::strcmp(e, "0") != 0;
    }();
    return on;
}

void log_launch(const char *entry, const pw_grid *g, pw_dtype dt, const TileCfg *c, const char *how) {
    if (!log_enabled()) return;
    static const char *names[] = {"f32", "f64", "bf16", "f16"};
    const char *dn = (dt >= PW_F32 && dt <= PW_F16) ? names[dt] : "?";
    if (c)
        std::fprintf(stderr, "pwadv: %s %lldx%lldx%lld halo %d %s tile (%d, %d, %d, %d, %d, %d) %s\n", entry,
                     (long long)g->nx, (long long)g->ny, (long long)g->nz, g->halo, dn, c->px, c->ry, c->zlen, c->wpb,
                     c->depth, c->share, how);
    else
        std::fprintf(stderr, "pwadv: %s %lldx%lldx%lld halo %d %s %s\n", entry, (long long)g->nx, (long long)g->ny,
                     (long long)g->nz, g->halo, dn, how);
}

namespace {

int64_t elem_size(pw_dtype dt) {
    switch (dt) {
        case PW_F32: return 4;
        case PW_F64: return 8;
        case PW_BF16: return 2;
        case PW_F16: return 2;
    }
    return 0;
}

// Element size of coefficients and outputs for a storage dtype.
int64_t compute_size(pw_dtype dt) { return dt == PW_F64 ? 8 : 4; }

struct Layout {
    int64_t in_sy, in_sz, out_sy, out_sz;
};

constexpr int64_t kMaxDim = int64_t(1) << 30;

pw_status check_grid(const pw_grid *g) {
    if (!g) return fail(PW_ERR_INVALID_ARG, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(PW_ERR_INVALID_ARG, "interior extents must be >= 1 (nx=%lld ny=%lld nz=%lld)",
                    (long long)g->nx, (long long)g->ny, (long long)g->nz);
    if (g->halo < 1) return fail(PW_ERR_INVALID_ARG, "halo must be >= 1 (depth-one stencil), got %d", g->halo);
    if (g->nx > kMaxDim || g->ny > kMaxDim || g->nz > kMaxDim || g->halo > 1024)
        return fail(PW_ERR_INVALID_ARG, "extent too large");
    if (g->nx * g->ny > (int64_t(1) << 40) / g->nz) return fail(PW_ERR_INVALID_ARG, "more than 2^40 points");
    return PW_OK;
}

pw_status resolve_layout(const pw_grid *g, const pw_layout *l, int64_t in_es, int64_t out_es, Layout *out) {
    const int64_t px = g->nx + 2 * g->halo, py = g->ny + 2 * g->halo;
    if (l) {
        *out = {l->in_sy, l->in_sz, l->out_sy, l->out_sz};
        if (out->in_sy < px) return fail(PW_ERR_INVALID_ARG, "in_sy %lld < nx+2h %lld", (long long)out->in_sy, (long long)px);
        if (out->in_sz / py < out->in_sy) return fail(PW_ERR_INVALID_ARG, "in_sz too small for in_sy*(ny+2h)");
        if (out->out_sy < g->nx) return fail(PW_ERR_INVALID_ARG, "out_sy %lld < nx", (long long)out->out_sy);
        if (out->out_sz / g->ny < out->out_sy) return fail(PW_ERR_INVALID_ARG, "out_sz too small for out_sy*ny");
    } else {
        *out = {px, px * py, g->nx, g->nx * g->ny};
    }
    // The kernels address within one z-plane with 32-bit byte offsets.
    if (out->in_sz * in_es >= (int64_t(1) << 31) || out->out_sz * out_es >= (int64_t(1) << 31))
        return fail(PW_ERR_UNSUPPORTED, "a z-plane larger than 2 GiB is not supported");
    return PW_OK;
}

struct Range {
    const char *name;
    uintptr_t lo, hi;
};

Range in_range(const char *name, const void *p, const pw_grid *g, const Layout &L, int64_t es) {
    const int64_t px = g->nx + 2 * g->halo, py = g->ny + 2 * g->halo, pz = g->nz + 2 * g->halo;
    const int64_t last = (pz - 1) * L.in_sz + (py - 1) * L.in_sy + (px - 1);
    return {name, reinterpret_cast<uintptr_t>(p), reinterpret_cast<uintptr_t>(p) + uintptr_t((last + 1) * es)};
}

Range out_range(const char *name, const void *p, const pw_grid *g, const Layout &L, int64_t es) {
    const int64_t last = (g->nz - 1) * L.out_sz + (g->ny - 1) * L.out_sy + (g->nx - 1);
    return {name, reinterpret_cast<uintptr_t>(p), reinterpret_cast<uintptr_t>(p) + uintptr_t((last + 1) * es)};
}

bool overlap(const Range &a, const Range &b) { return a.lo < b.hi && b.lo < a.hi; }

// Bytes [p, p + (last+1)*es) of an array whose last element is at offset `last`.
Range zspan(const char *name, const void *p, int64_t last, int64_t es) {
    const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return Range{name, lo, lo + uintptr_t((last + 1) * es)};
}

// Offset of the last interior output of a z-fastest array.
int64_t zfast_out_last(const pw_grid *g, int64_t osj, int64_t osi) {
    return (g->nx - 1) * osi + (g->ny - 1) * osj + (g->nz - 1);
}

// The kernels read the coefficient arrays through the scalar cache, which is
// only valid if nothing they write overlaps them.
pw_status check_coeffs_apart(const pw_coeffs *c, int64_t nz, int64_t cs, const Range *outs, int nout) {
    const void *p[4] = {c->tzc1, c->tzc2, c->tzd1, c->tzd2};
    const char *names[4] = {"tzc1", "tzc2", "tzd1", "tzd2"};
    for (int i = 0; i < 4; ++i) {
        const Range r{names[i], reinterpret_cast<uintptr_t>(p[i]), reinterpret_cast<uintptr_t>(p[i]) + uintptr_t(nz * cs)};
        for (int o = 0; o < nout; ++o)
            if (overlap(outs[o], r)) return fail(PW_ERR_INVALID_ARG, "%s overlaps coefficient array %s", outs[o].name, r.name);
    }
    return PW_OK;
}

pw_status check_aligned(const char *name, const void *p, int64_t es) {
    if (!p) return fail(PW_ERR_INVALID_ARG, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % uintptr_t(es))
        return fail(PW_ERR_INVALID_ARG, "%s is not aligned to its element size %lld", name, (long long)es);
    return PW_OK;
}

// The current device, after checking that one exists.
pw_status current_device(int *dev) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return fail(PW_ERR_NO_DEVICE, "no usable HIP device (%s)",
                    e == hipSuccess ? "device count 0" : hipGetErrorString(e));
    }
    e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return PW_OK;
}

pw_status check_on_device(const char *name, const void *p, int dev) {
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof at);
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PW_ERR_INVALID_ARG, "%s is not a device pointer", name);
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return fail(PW_ERR_INVALID_ARG, "%s is not device memory (memory type %d)", name, (int)at.type);
    if (at.device != dev)
        return fail(PW_ERR_INVALID_ARG, "%s lives on device %d, current device is %d", name, at.device, dev);
    return PW_OK;
}

#define PW_TRY(x)                            \
    do {                                     \
        pw_status st_ = (x);                 \
        if (st_ != PW_OK) return st_;        \
    } while (0)

}  // namespace

pw_status validate_forward(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                           const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                           void *su, void *sv, void *sw, FwdArgs *out) {
    PW_TRY(check_grid(grid));
    const int64_t es = elem_size(in_dtype);
    if (!es) return fail(PW_ERR_INVALID_ARG, "unknown dtype %d", (int)in_dtype);
    const int64_t cs = compute_size(in_dtype);
    Layout L;
    PW_TRY(resolve_layout(grid, layout, es, cs, &L));
    if (!coeffs) return fail(PW_ERR_INVALID_ARG, "coeffs is NULL");
    const char *names[] = {"u", "v", "w", "su", "sv", "sw", "tzc1", "tzc2", "tzd1", "tzd2"};
    const void *ptrs[] = {u, v, w, su, sv, sw, coeffs->tzc1, coeffs->tzc2, coeffs->tzd1, coeffs->tzd2};
    for (int i = 0; i < 10; ++i) PW_TRY(check_aligned(names[i], ptrs[i], i < 3 ? es : cs));
    const Range rin[3] = {in_range("u", u, grid, L, es), in_range("v", v, grid, L, es), in_range("w", w, grid, L, es)};
    const Range rout[3] = {out_range("su", su, grid, L, cs), out_range("sv", sv, grid, L, cs),
                           out_range("sw", sw, grid, L, cs)};
    for (const Range &o : rout) {
        for (const Range &i : rin)
            if (overlap(o, i)) return fail(PW_ERR_INVALID_ARG, "output %s overlaps input %s", o.name, i.name);
        for (const Range &o2 : rout)
            if (&o != &o2 && overlap(o, o2)) return fail(PW_ERR_INVALID_ARG, "outputs %s and %s overlap", o.name, o2.name);
    }
    PW_TRY(check_coeffs_apart(coeffs, grid->nz, cs, rout, 3));
    FwdArgs &a = *out;
    a.u = u; a.v = v; a.w = w;
    a.su = su; a.sv = sv; a.sw = sw;
    a.tzc1 = coeffs->tzc1; a.tzc2 = coeffs->tzc2; a.tzd1 = coeffs->tzd1; a.tzd2 = coeffs->tzd2;
    a.tcx = coeffs->tcx; a.tcy = coeffs->tcy;
    a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz; a.h = grid->halo;
    a.in_sy = L.in_sy; a.in_sz = L.in_sz; a.out_sy = L.out_sy; a.out_sz = L.out_sz;
    a.in_bytes = es;
    a.out_bytes = cs;
    return PW_OK;
}

pw_status check_forward_on_device(const FwdArgs &a) {
    const char *names[] = {"u", "v", "w", "su", "sv", "sw", "tzc1", "tzc2", "tzd1", "tzd2"};
    const void *ptrs[] = {a.u, a.v, a.w, a.su, a.sv, a.sw, a.tzc1, a.tzc2, a.tzd1, a.tzd2};
    int dev = 0;
    PW_TRY(current_device(&dev));
    for (int i = 0; i < 10; ++i) PW_TRY(check_on_device(names[i], ptrs[i], dev));
    return PW_OK;
}

void forward_ranges(const FwdArgs &a, uintptr_t (*in)[2], uintptr_t (*out)[2]) {
    const int64_t px = a.nx + 2 * a.h, py = a.ny + 2 * a.h, pz = a.nz + 2 * a.h;
    const int64_t ilast = (pz - 1) * a.in_sz + (py - 1) * a.in_sy + (px - 1);
    const int64_t olast = (a.nz - 1) * a.out_sz + (a.ny - 1) * a.out_sy + (a.nx - 1);
    const void *ip[3] = {a.u, a.v, a.w};
    const void *op[3] = {a.su, a.sv, a.sw};
    for (int i = 0; i < 3; ++i) {
        in[i][0] = reinterpret_cast<uintptr_t>(ip[i]);
        in[i][1] = in[i][0] + uintptr_t((ilast + 1) * a.in_bytes);
        out[i][0] = reinterpret_cast<uintptr_t>(op[i]);
        out[i][1] = out[i][0] + uintptr_t((olast + 1) * a.out_bytes);
    }
}

// Validation shared by the halo fill and fold: fills the launch operands.
pw_status validate_halo(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype, void *const fields[],
                        const pw_halo_modes modes[], int32_t nfields, HaloArgs *out) {
    PW_TRY(check_grid(grid));
    const int64_t es = elem_size(dtype);
    if (!es) return fail(PW_ERR_INVALID_ARG, "unknown dtype %d", int(dtype));
    if (!fields || !modes) return fail(PW_ERR_INVALID_ARG, "fields or modes is NULL");
    if (nfields < 1 || nfields > kMaxHaloFields)
        return fail(PW_ERR_INVALID_ARG, "nfields must be in 1..%d, got %d", kMaxHaloFields, nfields);
    const int64_t px = grid->nx + 2 * grid->halo, py = grid->ny + 2 * grid->halo;
    HaloArgs &a = *out;
    a.nf = nfields;
    a.es = int32_t(es);
    a.nx = grid->nx;
    a.ny = grid->ny;
    a.nz = grid->nz;
    a.h = grid->halo;
    a.sy = layout ? layout->in_sy : px;
    a.sz = layout ? layout->in_sz : px * py;
    if (a.sy < px) return fail(PW_ERR_INVALID_ARG, "in_sy %lld < nx+2h %lld", (long long)a.sy, (long long)px);
    if (a.sz / py < a.sy) return fail(PW_ERR_INVALID_ARG, "in_sz too small for in_sy*(ny+2h)");
    const int64_t n[3] = {grid->nx, grid->ny, grid->nz};
    const Layout L{a.sy, a.sz, grid->nx, grid->nx * grid->ny};
    Range r[kMaxHaloFields];
    static const char *const names[kMaxHaloFields] = {"fields[0]", "fields[1]", "fields[2]", "fields[3]",
                                                      "fields[4]", "fields[5]", "fields[6]", "fields[7]"};
    for (int f = 0; f < nfields; ++f) {
        PW_TRY(check_aligned(names[f], fields[f], es));
        const int32_t m[3] = {modes[f].x, modes[f].y, modes[f].z};
        for (int d = 0; d < 3; ++d) {
            if (m[d] < PW_HALO_KEEP || m[d] > PW_HALO_REFLECT_NEG)
                return fail(PW_ERR_INVALID_ARG, "modes[%d]: unknown halo mode %d", f, m[d]);
            if ((m[d] == PW_HALO_REFLECT || m[d] == PW_HALO_REFLECT_NEG) && n[d] < grid->halo)
                return fail(PW_ERR_INVALID_ARG, "modes[%d]: reflect on an axis of %lld cells needs halo <= %lld",
                            f, (long long)n[d], (long long)n[d]);
            a.mode[f][d] = m[d];
        }
        a.f[f] = fields[f];
        r[f] = in_range(names[f], fields[f], grid, L, es);
        for (int g = 0; g < f; ++g)
            if (overlap(r[f], r[g])) return fail(PW_ERR_INVALID_ARG, "%s overlaps %s", r[f].name, r[g].name);
    }
    int dev = 0;
    PW_TRY(current_device(&dev));
    for (int f = 0; f < nfields; ++f) PW_TRY(check_on_device(names[f], fields[f], dev));
    return PW_OK;
}

// The forward's launch shape: the caller's tile, else PWADV_TILE, else the
// tuned entry of the grid's class, else the default; `how` names the source
// (for PWADV_LOG).  No device work, so a bad PWADV_TILE fails before any.
pw_status forward_shape(const pw_grid *grid, const FwdArgs &a, pw_dtype dt, const pw_tile *tile, TileCfg *cfg,
                        const char **how) {
    if (tile) {
        *cfg = to_cfg(*tile);
        *how = "given";
        return PW_OK;
    }
    pw_tile t;
    const int e = env_forward_tile(&t);
    if (e < 0)
        return fail(PW_ERR_INVALID_ARG,
                    "PWADV_TILE=\"%s\" is not a launch shape (cols_per_lane x rows_per_strip x zlen "
                    "[x waves_per_group [x prefetch [x share_rows]]])",
                    std::getenv("PWADV_TILE"));
    if (e > 0) {
        if (!tile_supported(to_cfg(t), dt))
            return fail(PW_ERR_INVALID_ARG, "PWADV_TILE=\"%s\" is not a forward shape for this storage type",
                        std::getenv("PWADV_TILE"));
        *cfg = to_cfg(t);
        *how = "PWADV_TILE";
        return PW_OK;
    }
    if (lookup_tuned(TuneKind::Forward, grid, dt, cfg)) {
        *how = "tuned";
        return PW_OK;
    }
    *cfg = default_forward_tile(a, dt);
    *how = "default";
    return PW_OK;
}

// Forward with optional boundary rules (bc, NULL: read the stored halo) and
// optional fused epilogue (ep, NULL: out = F): validation and launch.
pw_status advect_general(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype, const void *u,
                         const void *v, const void *w, const pw_coeffs *coeffs, const pw_halo_modes *bc,
                         const pw_epilogue *ep, void *su, void *sv, void *sw, const pw_tile *tile,
                         void *hip_stream) {
    FwdArgs a;
    PW_TRY(validate_forward(grid, layout, in_dtype, u, v, w, coeffs, su, sv, sw, &a));
    if (tile && !tile_supported(to_cfg(*tile), in_dtype))
        return fail(PW_ERR_INVALID_ARG,
                    "unsupported forward tile cols=%d rows=%d zlen=%d waves=%d prefetch=%d share_rows=%d",
                    tile->cols_per_lane, tile->rows_per_strip, tile->zlen, tile->waves_per_group, tile->prefetch,
                    tile->share_rows);
    TileCfg cfg;
    const char *how = "given";
    PW_TRY(forward_shape(grid, a, in_dtype, tile, &cfg, &how));
    if (bc) {
        // bc[f] = rules of field f (u, v, w).  A depth-one read of a halo cell
        // goes to its periodic source or to the nearest interior cell (which
        // is also the mirror image of the cells next to the face); ZERO and
        // REFLECT_NEG then change the value.  The remapping is shared by the
        // three fields, so per axis they must agree on it.
        const int64_t n[3] = {grid->nx, grid->ny, grid->nz};
        int32_t addr[3] = {-1, -1, -1};
        uint32_t bcv = 0;
        for (int f = 0; f < 3; ++f) {
            const int32_t m[3] = {bc[f].x, bc[f].y, bc[f].z};
            for (int d = 0; d < 3; ++d) {
                if (m[d] < PW_HALO_KEEP || m[d] > PW_HALO_REFLECT_NEG)
                    return fail(PW_ERR_INVALID_ARG, "unknown boundary rule %d (field %c, axis %c)", m[d], "uvw"[f],
                                "xyz"[d]);
                if ((m[d] == PW_HALO_REFLECT || m[d] == PW_HALO_REFLECT_NEG) && n[d] < grid->halo)
                    return fail(PW_ERR_INVALID_ARG, "reflect on axis %c needs at least %d interior cells",
                                "xyz"[d], grid->halo);
                const int32_t cls = m[d] == PW_HALO_KEEP ? PW_HALO_KEEP
                                    : m[d] == PW_HALO_PERIODIC ? PW_HALO_PERIODIC : PW_HALO_COPY;
                if (addr[d] >= 0 && addr[d] != cls)
                    return fail(PW_ERR_UNSUPPORTED,
                                "axis %c: u, v and w must all keep, all be periodic, or all use nearest-cell rules "
                                "(copy, zero, reflect, reflect_neg)", "xyz"[d]);
                addr[d] = cls;
                const uint32_t code = m[d] == PW_HALO_REFLECT_NEG ? 1u : (m[d] == PW_HALO_ZERO ? 2u : 0u);
                bcv |= code << (8 * d + 2 * f);
            }
        }
        a.bcx = addr[0];
        a.bcy = addr[1];
        a.bcz = addr[2];
        a.bcv = bcv;
    }
    int dev = 0;
    if (ep) {
        // the addends: output layout, compute type; each either is its output
        // (accumulation in place) or overlaps no output at all (inputs may be
        // overlapped: they are only read)
        const int64_t cs = a.out_bytes;
        Layout L;
        PW_TRY(resolve_layout(grid, layout, a.in_bytes, cs, &L));
        const char *cn[3] = {"cu", "cv", "cw"};
        const void *cp[3] = {ep->cu, ep->cv, ep->cw};
        void *op[3] = {su, sv, sw};
        const Range rout[3] = {out_range("su", su, grid, L, cs), out_range("sv", sv, grid, L, cs),
                               out_range("sw", sw, grid, L, cs)};
        for (int i = 0; i < 3; ++i) {
            PW_TRY(check_aligned(cn[i], cp[i], cs));
            const Range rc = out_range(cn[i], cp[i], grid, L, cs);
            for (int o = 0; o < 3; ++o) {
                if (o == i && cp[i] == op[o]) continue;   // in place
                if (overlap(rc, rout[o]))
                    return fail(PW_ERR_INVALID_ARG, "%s overlaps output %s (only %s itself may be given)", cn[i],
                                rout[o].name, rout[i].name);
            }
        }
        if (!std::isfinite(ep->alpha)) return fail(PW_ERR_INVALID_ARG, "alpha is not finite");
        PW_TRY(check_forward_on_device(a));
        PW_TRY(current_device(&dev));
        for (int i = 0; i < 3; ++i) PW_TRY(check_on_device(cn[i], cp[i], dev));
        a.epilogue = true;
        a.cu = ep->cu; a.cv = ep->cv; a.cw = ep->cw;
        a.alpha = ep->alpha;
    } else {
        PW_TRY(check_forward_on_device(a));
    }
    log_launch(bc ? "pw_advect_bc" : "pw_advect_epilogue", grid, in_dtype, &cfg, how);
    return launch_forward(a, in_dtype, cfg, static_cast<hipStream_t>(hip_stream));
}

}  // namespace pw

using namespace pw;

extern "C" {

const char *pw_version(void) { return "libpwadv 0.1.0 (gfx950)"; }

const char *pw_last_error(void) { return g_err; }

pw_status pw_advect(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                    const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                    void *su, void *sv, void *sw, void *hip_stream) {
    return pw_advect_ex(grid, layout, in_dtype, u, v, w, coeffs, su, sv, sw, nullptr, hip_stream);
}

pw_status pw_advect_ex(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                       const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                       void *su, void *sv, void *sw, const pw_tile *tile, void *hip_stream) {
    g_err[0] = 0;
    FwdArgs a;
    PW_TRY(validate_forward(grid, layout, in_dtype, u, v, w, coeffs, su, sv, sw, &a));
    if (tile && !tile_supported(to_cfg(*tile), in_dtype))
        return fail(PW_ERR_INVALID_ARG,
                    "unsupported forward tile cols=%d rows=%d zlen=%d waves=%d prefetch=%d share_rows=%d",
                    tile->cols_per_lane, tile->rows_per_strip, tile->zlen, tile->waves_per_group, tile->prefetch,
                    tile->share_rows);
    TileCfg cfg;
    const char *how = "given";
    PW_TRY(forward_shape(grid, a, in_dtype, tile, &cfg, &how));
    PW_TRY(check_forward_on_device(a));
    log_launch("pw_advect", grid, in_dtype, &cfg, how);
    return launch_forward(a, in_dtype, cfg, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_advect_epilogue(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                             const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                             const pw_epilogue *ep, void *su, void *sv, void *sw, const pw_tile *tile,
                             void *hip_stream) {
    g_err[0] = 0;
    if (!ep) return fail(PW_ERR_INVALID_ARG, "epilogue is NULL");
    return advect_general(grid, layout, in_dtype, u, v, w, coeffs, nullptr, ep, su, sv, sw, tile, hip_stream);
}

pw_status pw_advect_bc(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype, const void *u,
                       const void *v, const void *w, const pw_coeffs *coeffs, const pw_halo_modes bc[3],
                       const pw_epilogue *ep, void *su, void *sv, void *sw, const pw_tile *tile, void *hip_stream) {
    g_err[0] = 0;
    if (!bc) return fail(PW_ERR_INVALID_ARG, "bc is NULL");
    return advect_general(grid, layout, in_dtype, u, v, w, coeffs, bc, ep, su, sv, sw, tile, hip_stream);
}

pw_status pw_advect_tangent(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                            const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                            const void *du, const void *dv, const void *dw,
                            void *tu, void *tv, void *tw, void *hip_stream) {
    return pw_advect_tangent_ex(grid, layout, dtype, u, v, w, coeffs, du, dv, dw, tu, tv, tw, nullptr, hip_stream);
}

pw_status pw_advect_tangent_ex(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                               const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                               const void *du, const void *dv, const void *dw,
                               void *tu, void *tv, void *tw, const pw_tile *tile, void *hip_stream) {
    g_err[0] = 0;
    PW_TRY(check_grid(grid));
    if (dtype != PW_F32 && dtype != PW_F64) {
        if (elem_size(dtype)) return fail(PW_ERR_UNSUPPORTED, "tangent supports PW_F32 and PW_F64 only");
        return fail(PW_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    }
    TanArgs a;
    // values, coefficients and outputs exactly as for the forward operator
    PW_TRY(validate_forward(grid, layout, dtype, u, v, w, coeffs, tu, tv, tw, &a.f));
    const int64_t es = elem_size(dtype);
    Layout L;
    PW_TRY(resolve_layout(grid, layout, es, es, &L));
    const char *names[] = {"du", "dv", "dw"};
    const void *ptrs[] = {du, dv, dw};
    for (int i = 0; i < 3; ++i) PW_TRY(check_aligned(names[i], ptrs[i], es));
    const Range rdir[3] = {in_range("du", du, grid, L, es), in_range("dv", dv, grid, L, es),
                           in_range("dw", dw, grid, L, es)};
    const Range rout[3] = {out_range("tu", tu, grid, L, es), out_range("tv", tv, grid, L, es),
                           out_range("tw", tw, grid, L, es)};
    for (const Range &o : rout)
        for (const Range &i : rdir)
            if (overlap(o, i)) return fail(PW_ERR_INVALID_ARG, "output %s overlaps direction %s", o.name, i.name);
    if (tile && !tangent_tile_supported(to_cfg(*tile), dtype))
        return fail(PW_ERR_INVALID_ARG, "unsupported tangent tile cols=%d rows=%d zlen=%d waves=%d prefetch=%d",
                    tile->cols_per_lane, tile->rows_per_strip, tile->zlen, tile->waves_per_group, tile->prefetch);
    PW_TRY(check_forward_on_device(a.f));
    int dev = 0;
    PW_TRY(current_device(&dev));
    for (int i = 0; i < 3; ++i) PW_TRY(check_on_device(names[i], ptrs[i], dev));
    a.du = du;
    a.dv = dv;
    a.dw = dw;
    TileCfg cfg;
    const char *how = "given";
    if (tile)
        cfg = to_cfg(*tile);
    else if (lookup_tuned(TuneKind::Tangent, grid, dtype, &cfg))
        how = "tuned";
    else
        cfg = default_tangent_tile(a, dtype), how = "default";
    log_launch("pw_advect_tangent", grid, dtype, &cfg, how);
    return launch_tangent(a, dtype, cfg, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_advect_coeff_grad_workspace(const pw_grid *grid, pw_dtype dtype, int64_t *bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(PW_ERR_INVALID_ARG, "bytes is NULL");
    PW_TRY(check_grid(grid));
    if (dtype != PW_F32 && dtype != PW_F64) {
        if (elem_size(dtype)) return fail(PW_ERR_UNSUPPORTED, "coefficient gradients support PW_F32 and PW_F64 only");
        return fail(PW_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    }
    *bytes = coeff_grad_workspace_bytes(*grid, dtype);
    return PW_OK;
}

namespace {

// Validation shared by both coefficient-gradient entry points.  With
// workspace == NULL (the library's own scratch) only the caller's arrays are
// checked, and the scratch's size is checked against the need instead.
pw_status check_coeff_grad(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                           const void *u, const void *v, const void *w,
                           const void *gsu, const void *gsv, const void *gsw,
                           double *grad, void *workspace, int64_t workspace_bytes, Layout *Lout,
                           bool device = true) {
    int64_t need = 0;
    PW_TRY(pw_advect_coeff_grad_workspace(grid, dtype, &need));
    const int64_t es = elem_size(dtype);
    Layout L;
    PW_TRY(resolve_layout(grid, layout, es, es, &L));
    const bool own = workspace == nullptr;
    const int nptr = own ? 7 : 8;
    const char *names[] = {"u", "v", "w", "gsu", "gsv", "gsw", "grad", "workspace"};
    const void *ptrs[] = {u, v, w, gsu, gsv, gsw, grad, workspace};
    if (own && need > kCoeffGradScratchBytes)
        return fail(PW_ERR_UNSUPPORTED,
                    "grid needs %lld bytes of partials, beyond the %lld-byte static scratch: "
                    "use pw_advect_coeff_grad with a workspace",
                    (long long)need, (long long)kCoeffGradScratchBytes);
    for (int i = 0; i < 6; ++i) PW_TRY(check_aligned(names[i], ptrs[i], es));
    for (int i = 6; i < nptr; ++i) PW_TRY(check_aligned(names[i], ptrs[i], 8));
    if (!own && workspace_bytes < need)
        return fail(PW_ERR_INVALID_ARG, "workspace of %lld bytes is smaller than the %lld needed",
                    (long long)workspace_bytes, (long long)need);
    const Range rin[6] = {in_range("u", u, grid, L, es), in_range("v", v, grid, L, es), in_range("w", w, grid, L, es),
                          out_range("gsu", gsu, grid, L, es), out_range("gsv", gsv, grid, L, es),
                          out_range("gsw", gsw, grid, L, es)};
    const uintptr_t gb = reinterpret_cast<uintptr_t>(grad), wb = reinterpret_cast<uintptr_t>(workspace);
    const Range rout[2] = {{"grad", gb, gb + uintptr_t((6 * grid->nz + 2) * 8)}, {"workspace", wb, wb + uintptr_t(need)}};
    for (int o = 0; o < nptr - 6; ++o)
        for (const Range &i : rin)
            if (overlap(rout[o], i)) return fail(PW_ERR_INVALID_ARG, "%s overlaps %s", rout[o].name, i.name);
    if (!own && overlap(rout[0], rout[1])) return fail(PW_ERR_INVALID_ARG, "grad overlaps workspace");
    *Lout = L;
    if (!device) return PW_OK;
    int dev = 0;
    PW_TRY(current_device(&dev));
    for (int i = 0; i < nptr; ++i) PW_TRY(check_on_device(names[i], ptrs[i], dev));
    return PW_OK;
}

}  // namespace

}  // extern "C"

namespace pw {
namespace {

// Launch shape of every coefficient-gradient pass, fixed by the grid's size
// alone, so that the partials -- and the gradients -- are the same bit for
// bit whether the wind gradients are computed with them or not.  Measured on
// MI355X (256x256x128 FP32, the three adjoint modes over rows per strip,
// z-chunks, wavefronts per workgroup and prefetch depth): four-row strips
// (FP64: one row, for registers), one wavefront per workgroup, and the march
// cut into as many z-chunks as keep the wavefronts within one round of the
// chip's 2048 slots (these kernels hold about 220 VGPRs: two wavefronts per
// SIMD).  One round more with a short tail costs a quarter: 2275 wavefronts
// took 139 us where 1950 took 113 us.
TileCfg coeff_grad_tile(const pw_grid *grid, pw_dtype dtype) {
    TileCfg c;
    c.px = 1;
    c.ry = dtype == PW_F64 ? 1 : 4;
    c.wpb = 1;
    c.depth = 1;
    c.share = 0;
    const int64_t pz = grid->nz + 2 * grid->halo;
    const int64_t strips = adjoint_strips(*grid, c.ry);
    int64_t chunks = 2048 / strips;
    if (chunks < 1) chunks = 1;
    int64_t zl = (pz + chunks - 1) / chunks;
    if (zl < 8) zl = 8;
    if (zl > pz) zl = pz;
    c.zlen = static_cast<int>(zl);
    return c;
}

AdjArgs coeff_grad_args(const pw_grid *grid, const Layout &L, const void *u, const void *v, const void *w,
                        const void *gsu, const void *gsv, const void *gsw) {
    AdjArgs a{};
    a.u = u; a.v = v; a.w = w;
    a.gsu = gsu; a.gsv = gsv; a.gsw = gsw;
    a.gu = a.gv = a.gw = nullptr;
    a.tzc1 = a.tzc2 = a.tzd1 = a.tzd2 = nullptr;
    a.tcx = a.tcy = 0.0;
    a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz; a.h = grid->halo;
    a.in_sy = L.in_sy; a.in_sz = L.in_sz; a.out_sy = L.out_sy; a.out_sz = L.out_sz;
    return a;
}

pw_status run_coeff_grad(const pw_grid *grid, pw_dtype dtype, const AdjArgs &a, bool grads, double *grad,
                         void *workspace, hipStream_t s) {
    const TileCfg cfg = coeff_grad_tile(grid, dtype);
    log_launch(grads ? "pw_advect_adjoint_coeff_grad" : "pw_advect_coeff_grad", grid, dtype, &cfg, "shape rule");
    double *ws = static_cast<double *>(workspace);
    PW_TRY(launch_adjoint_mode(a, dtype, cfg, grads, ws, s));
    return launch_coeff_grad_reduce(ws, adjoint_strips(*grid, cfg.ry), grad, grid->nz, s);
}

}  // namespace
}  // namespace pw

extern "C" {

pw_status pw_advect_coeff_grad_static(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                                      const void *u, const void *v, const void *w,
                                      const void *gsu, const void *gsv, const void *gsw,
                                      double *grad, void *hip_stream) {
    g_err[0] = 0;
    Layout L;
    PW_TRY(check_coeff_grad(grid, layout, dtype, u, v, w, gsu, gsv, gsw, grad, nullptr, 0, &L));
    void *ws = nullptr;
    PW_TRY(coeff_grad_scratch(&ws));
    const AdjArgs a = coeff_grad_args(grid, L, u, v, w, gsu, gsv, gsw);
    return run_coeff_grad(grid, dtype, a, false, grad, ws, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_advect_coeff_grad(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                               const void *u, const void *v, const void *w,
                               const void *gsu, const void *gsv, const void *gsw,
                               double *grad, void *workspace, int64_t workspace_bytes, void *hip_stream) {
    g_err[0] = 0;
    if (!workspace) return fail(PW_ERR_INVALID_ARG, "workspace is NULL");
    Layout L;
    PW_TRY(check_coeff_grad(grid, layout, dtype, u, v, w, gsu, gsv, gsw, grad, workspace, workspace_bytes, &L));
    const AdjArgs a = coeff_grad_args(grid, L, u, v, w, gsu, gsv, gsw);
    return run_coeff_grad(grid, dtype, a, false, grad, workspace, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_advect_adjoint(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                            const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                            const void *gsu, const void *gsv, const void *gsw,
                            void *gu, void *gv, void *gw, void *hip_stream) {
    return pw_advect_adjoint_ex(grid, layout, dtype, u, v, w, coeffs, gsu, gsv, gsw, gu, gv, gw, nullptr,
                                hip_stream);
}

namespace {

// Validation of the adjoint's operands; fills `a` and the resolved layout.
pw_status check_adjoint(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                        const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                        const void *gsu, const void *gsv, const void *gsw,
                        void *gu, void *gv, void *gw, const pw_tile *tile, AdjArgs *aout, Layout *Lout,
                        bool device = true) {
    PW_TRY(check_grid(grid));
    if (dtype != PW_F32 && dtype != PW_F64) {
        if (elem_size(dtype)) return fail(PW_ERR_UNSUPPORTED, "adjoint supports PW_F32 and PW_F64 only");
        return fail(PW_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    }
    const int64_t es = elem_size(dtype);
    Layout L;
    PW_TRY(resolve_layout(grid, layout, es, es, &L));
    if (!coeffs) return fail(PW_ERR_INVALID_ARG, "coeffs is NULL");
    const char *names[] = {"u", "v", "w", "gsu", "gsv", "gsw", "gu", "gv", "gw", "tzc1", "tzc2", "tzd1", "tzd2"};
    const void *ptrs[] = {u, v, w, gsu, gsv, gsw, gu, gv, gw, coeffs->tzc1, coeffs->tzc2, coeffs->tzd1, coeffs->tzd2};
    for (int i = 0; i < 13; ++i) PW_TRY(check_aligned(names[i], ptrs[i], es));
    const Range rin[6] = {in_range("u", u, grid, L, es), in_range("v", v, grid, L, es), in_range("w", w, grid, L, es),
                          out_range("gsu", gsu, grid, L, es), out_range("gsv", gsv, grid, L, es),
                          out_range("gsw", gsw, grid, L, es)};
    const Range rout[3] = {in_range("gu", gu, grid, L, es), in_range("gv", gv, grid, L, es),
                           in_range("gw", gw, grid, L, es)};
    for (const Range &o : rout) {
        for (const Range &i : rin)
            if (overlap(o, i)) return fail(PW_ERR_INVALID_ARG, "gradient %s overlaps %s", o.name, i.name);
        for (const Range &o2 : rout)
            if (&o != &o2 && overlap(o, o2)) return fail(PW_ERR_INVALID_ARG, "gradients %s and %s overlap", o.name, o2.name);
    }
    PW_TRY(check_coeffs_apart(coeffs, grid->nz, es, rout, 3));
    if (tile && !adjoint_tile_supported(to_cfg(*tile)))
        return fail(PW_ERR_INVALID_ARG, "unsupported adjoint tile cols=%d rows=%d zlen=%d waves=%d prefetch=%d",
                    tile->cols_per_lane, tile->rows_per_strip, tile->zlen, tile->waves_per_group, tile->prefetch);
    if (device) {
        int dev = 0;
        PW_TRY(current_device(&dev));
        for (int i = 0; i < 13; ++i) PW_TRY(check_on_device(names[i], ptrs[i], dev));
    }

    AdjArgs a;
    a.u = u; a.v = v; a.w = w;
    a.gsu = gsu; a.gsv = gsv; a.gsw = gsw;
    a.gu = gu; a.gv = gv; a.gw = gw;
    a.tzc1 = coeffs->tzc1; a.tzc2 = coeffs->tzc2; a.tzd1 = coeffs->tzd1; a.tzd2 = coeffs->tzd2;
    a.tcx = coeffs->tcx; a.tcy = coeffs->tcy;
    a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz; a.h = grid->halo;
    a.in_sy = L.in_sy; a.in_sz = L.in_sz; a.out_sy = L.out_sy; a.out_sz = L.out_sz;
    *aout = a;
    *Lout = L;
    return PW_OK;
}

}  // namespace

pw_status pw_advect_adjoint_ex(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                               const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                               const void *gsu, const void *gsv, const void *gsw,
                               void *gu, void *gv, void *gw, const pw_tile *tile, void *hip_stream) {
    g_err[0] = 0;
    AdjArgs a;
    Layout L;
    PW_TRY(check_adjoint(grid, layout, dtype, u, v, w, coeffs, gsu, gsv, gsw, gu, gv, gw, tile, &a, &L));
    TileCfg cfg;
    const char *how = "given";
    if (tile)
        cfg = to_cfg(*tile);
    else if (lookup_tuned(TuneKind::Adjoint, grid, dtype, &cfg))
        how = "tuned";
    else
        cfg = default_adjoint_tile(a, dtype), how = "default";
    log_launch("pw_advect_adjoint", grid, dtype, &cfg, how);
    return launch_adjoint(a, dtype, cfg, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_advect_adjoint_coeff_grad(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                                       const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                                       const void *gsu, const void *gsv, const void *gsw,
                                       void *gu, void *gv, void *gw, double *grad, void *workspace,
                                       int64_t workspace_bytes, void *hip_stream) {
    g_err[0] = 0;
    if (!workspace) return fail(PW_ERR_INVALID_ARG, "workspace is NULL");
    // every argument check first, then the device checks (so that the checks
    // can be tested without a GPU)
    AdjArgs a;
    Layout L;
    PW_TRY(check_adjoint(grid, layout, dtype, u, v, w, coeffs, gsu, gsv, gsw, gu, gv, gw, nullptr, &a, &L, false));
    Layout L2;
    PW_TRY(check_coeff_grad(grid, layout, dtype, u, v, w, gsu, gsv, gsw, grad, workspace, workspace_bytes, &L2,
                            false));
    // grad and the workspace also stay apart from the wind gradients
    const int64_t es = elem_size(dtype);
    int64_t need = 0;
    PW_TRY(pw_advect_coeff_grad_workspace(grid, dtype, &need));
    const uintptr_t gb = reinterpret_cast<uintptr_t>(grad), wb = reinterpret_cast<uintptr_t>(workspace);
    const Range rcg[2] = {{"grad", gb, gb + uintptr_t((6 * grid->nz + 2) * 8)}, {"workspace", wb, wb + uintptr_t(need)}};
    const Range rg[3] = {in_range("gu", gu, grid, L, es), in_range("gv", gv, grid, L, es),
                         in_range("gw", gw, grid, L, es)};
    for (const Range &c : rcg)
        for (const Range &o : rg)
            if (overlap(c, o)) return fail(PW_ERR_INVALID_ARG, "%s overlaps %s", c.name, o.name);
    PW_TRY(check_adjoint(grid, layout, dtype, u, v, w, coeffs, gsu, gsv, gsw, gu, gv, gw, nullptr, &a, &L));
    PW_TRY(check_coeff_grad(grid, layout, dtype, u, v, w, gsu, gsv, gsw, grad, workspace, workspace_bytes, &L2));
    return run_coeff_grad(grid, dtype, a, true, grad, workspace, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

namespace pw {
namespace {

// Validation shared by the z-fastest entry points: fills the launch operands
// (strides in FwdArgs' row / plane fields) and the output byte ranges.
pw_status validate_zfast(const pw_grid *grid, const pw_layout_zfast *layout, pw_dtype in_dtype, const void *u,
                         const void *v, const void *w, const pw_coeffs *coeffs, void *su, void *sv, void *sw,
                         const pw_tile *tile, FwdArgs *out, Range (&rout)[3]) {
    PW_TRY(check_grid(grid));
    const int64_t es = elem_size(in_dtype);
    if (!es) return fail(PW_ERR_INVALID_ARG, "unknown dtype %d", (int)in_dtype);
    const int64_t cs = compute_size(in_dtype);
    if (!coeffs) return fail(PW_ERR_INVALID_ARG, "coeffs is NULL");
    const int64_t h = grid->halo, px = grid->nx + 2 * h, py = grid->ny + 2 * h, pz = grid->nz + 2 * h;
    int64_t isj = pz, isi = py * pz, osj = grid->nz, osi = grid->ny * grid->nz;
    if (layout) {
        isj = layout->in_sj;
        isi = layout->in_si;
        osj = layout->out_sj;
        osi = layout->out_si;
        if (isj < pz) return fail(PW_ERR_INVALID_ARG, "in_sj %lld < nz+2h %lld", (long long)isj, (long long)pz);
        if (isi / py < isj) return fail(PW_ERR_INVALID_ARG, "in_si too small for in_sj*(ny+2h)");
        if (osj < grid->nz) return fail(PW_ERR_INVALID_ARG, "out_sj %lld < nz", (long long)osj);
        if (osi / grid->ny < osj) return fail(PW_ERR_INVALID_ARG, "out_si too small for out_sj*ny");
    }
    if (isi * es >= (int64_t(1) << 31) || osi * cs >= (int64_t(1) << 31))
        return fail(PW_ERR_UNSUPPORTED, "an x-plane larger than 2 GiB is not supported");
    const char *names[] = {"u", "v", "w", "su", "sv", "sw", "tzc1", "tzc2", "tzd1", "tzd2"};
    const void *ptrs[] = {u, v, w, su, sv, sw, coeffs->tzc1, coeffs->tzc2, coeffs->tzd1, coeffs->tzd2};
    for (int i = 0; i < 10; ++i) PW_TRY(check_aligned(names[i], ptrs[i], i < 3 ? es : cs));
    const int64_t ilast = (px - 1) * isi + (py - 1) * isj + (pz - 1);
    const Range rin[3] = {zspan("u", u, ilast, es), zspan("v", v, ilast, es), zspan("w", w, ilast, es)};
    const int64_t olast = zfast_out_last(grid, osj, osi);
    rout[0] = zspan("su", su, olast, cs);
    rout[1] = zspan("sv", sv, olast, cs);
    rout[2] = zspan("sw", sw, olast, cs);
    for (const Range &o : rout) {
        for (const Range &i : rin)
            if (overlap(o, i)) return fail(PW_ERR_INVALID_ARG, "output %s overlaps input %s", o.name, i.name);
        for (const Range &o2 : rout)
            if (&o != &o2 && overlap(o, o2)) return fail(PW_ERR_INVALID_ARG, "outputs %s and %s overlap", o.name, o2.name);
    }
    PW_TRY(check_coeffs_apart(coeffs, grid->nz, cs, rout, 3));
    if (tile && !zfast_tile_supported(to_cfg(*tile), in_dtype))
        return fail(PW_ERR_INVALID_ARG, "unsupported z-fastest tile levels=%d rows=%d xlen=%d waves=%d prefetch=%d",
                    tile->cols_per_lane, tile->rows_per_strip, tile->zlen, tile->waves_per_group, tile->prefetch);
    FwdArgs &a = *out;
    a.u = u; a.v = v; a.w = w;
    a.su = su; a.sv = sv; a.sw = sw;
    a.tzc1 = coeffs->tzc1; a.tzc2 = coeffs->tzc2; a.tzd1 = coeffs->tzd1; a.tzd2 = coeffs->tzd2;
    a.tcx = coeffs->tcx; a.tcy = coeffs->tcy;
    a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz; a.h = grid->halo;
    a.in_sy = isj; a.in_sz = isi; a.out_sy = osj; a.out_sz = osi;
    a.in_bytes = es;
    a.out_bytes = cs;
    return PW_OK;
}

pw_status launch_zfast_tuned(const pw_grid *grid, pw_dtype in_dtype, const FwdArgs &a, const pw_tile *tile,
                             void *hip_stream) {
    PW_TRY(check_forward_on_device(a));
    TileCfg cfg;
    const char *how = "given";
    if (tile)
        cfg = to_cfg(*tile);
    else if (lookup_tuned(TuneKind::Zfast, grid, in_dtype, &cfg))
        how = "tuned";
    else
        cfg = default_zfast_tile(a, in_dtype), how = "default";
    log_launch(a.epilogue ? "pw_advect_zfast_epilogue" : "pw_advect_zfast", grid, in_dtype, &cfg, how);
    return launch_zfast(a, in_dtype, cfg, static_cast<hipStream_t>(hip_stream));
}

}  // namespace
}  // namespace pw

extern "C" {

pw_status pw_advect_zfast(const pw_grid *grid, const pw_layout_zfast *layout, pw_dtype in_dtype,
                          const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                          void *su, void *sv, void *sw, const pw_tile *tile, void *hip_stream) {
    g_err[0] = 0;
    FwdArgs a;
    Range rout[3];
    PW_TRY(validate_zfast(grid, layout, in_dtype, u, v, w, coeffs, su, sv, sw, tile, &a, rout));
    return launch_zfast_tuned(grid, in_dtype, a, tile, hip_stream);
}

pw_status pw_advect_zfast_epilogue(const pw_grid *grid, const pw_layout_zfast *layout, pw_dtype in_dtype,
                                   const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                                   const pw_epilogue *ep, void *su, void *sv, void *sw, const pw_tile *tile,
                                   void *hip_stream) {
    g_err[0] = 0;
    if (!ep) return fail(PW_ERR_INVALID_ARG, "epilogue is NULL");
    FwdArgs a;
    Range rout[3];
    PW_TRY(validate_zfast(grid, layout, in_dtype, u, v, w, coeffs, su, sv, sw, tile, &a, rout));
    // the addends: output layout, compute type; each either is its output
    // (accumulation in place) or overlaps no output at all
    const int64_t cs = a.out_bytes;
    const int64_t olast = zfast_out_last(grid, a.out_sy, a.out_sz);
    const char *cn[3] = {"cu", "cv", "cw"};
    const void *cp[3] = {ep->cu, ep->cv, ep->cw};
    void *op[3] = {su, sv, sw};
    for (int i = 0; i < 3; ++i) {
        PW_TRY(check_aligned(cn[i], cp[i], cs));
        const Range rc = zspan(cn[i], cp[i], olast, cs);
        for (int o = 0; o < 3; ++o) {
            if (o == i && cp[i] == op[o]) continue;   // in place
            if (overlap(rc, rout[o]))
                return fail(PW_ERR_INVALID_ARG, "%s overlaps output %s (only %s itself may be given)", cn[i],
                            rout[o].name, rout[i].name);
        }
    }
    if (!std::isfinite(ep->alpha)) return fail(PW_ERR_INVALID_ARG, "alpha is not finite");
    int dev = 0;
    PW_TRY(current_device(&dev));
    for (int i = 0; i < 3; ++i) PW_TRY(check_on_device(cn[i], cp[i], dev));
    a.epilogue = true;
    a.cu = ep->cu; a.cv = ep->cv; a.cw = ep->cw;
    a.alpha = ep->alpha;
    return launch_zfast_tuned(grid, in_dtype, a, tile, hip_stream);
}

pw_status pw_halo_fill(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype, void *const fields[],
                       const pw_halo_modes modes[], int32_t nfields, void *hip_stream) {
    g_err[0] = 0;
    HaloArgs a{};
    PW_TRY(validate_halo(grid, layout, dtype, fields, modes, nfields, &a));
    log_launch("pw_halo_fill", grid, dtype, nullptr, nfields == 1 ? "1 field" : "several fields");
    return launch_halo(a, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_halo_fold(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype, void *const fields[],
                       const pw_halo_modes modes[], int32_t nfields, void *hip_stream) {
    g_err[0] = 0;
    if (dtype != PW_F32 && dtype != PW_F64)
        return fail(PW_ERR_UNSUPPORTED, "the halo fold (a gradient operation) supports PW_F32 and PW_F64 only");
    HaloArgs a{};
    PW_TRY(validate_halo(grid, layout, dtype, fields, modes, nfields, &a));
    log_launch("pw_halo_fold", grid, dtype, nullptr, nfields == 1 ? "1 field" : "several fields");
    return launch_halo_fold(a, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_stream_copy(const void *src, void *dst, int64_t nbytes, void *hip_stream) {
    g_err[0] = 0;
    if (!src || !dst) return fail(PW_ERR_INVALID_ARG, "NULL pointer");
    if (nbytes <= 0 || nbytes % 16) return fail(PW_ERR_INVALID_ARG, "nbytes must be a positive multiple of 16");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
        return fail(PW_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    const Range a{"src", reinterpret_cast<uintptr_t>(src), reinterpret_cast<uintptr_t>(src) + uintptr_t(nbytes)};
    const Range b{"dst", reinterpret_cast<uintptr_t>(dst), reinterpret_cast<uintptr_t>(dst) + uintptr_t(nbytes)};
    if (overlap(a, b)) return fail(PW_ERR_INVALID_ARG, "src and dst overlap");
    int dev = 0;
    PW_TRY(current_device(&dev));
    PW_TRY(check_on_device("src", src, dev));
    PW_TRY(check_on_device("dst", dst, dev));
    return launch_copy(src, dst, nbytes, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_stream_copy3(const void *const src[3], void *const dst[3], int64_t nbytes, void *hip_stream) {
    g_err[0] = 0;
    if (!src || !dst) return fail(PW_ERR_INVALID_ARG, "NULL pointer array");
    if (nbytes <= 0 || nbytes % 16) return fail(PW_ERR_INVALID_ARG, "nbytes must be a positive multiple of 16");
    const void *p[6] = {src[0], src[1], src[2], dst[0], dst[1], dst[2]};
    const char *names[6] = {"src[0]", "src[1]", "src[2]", "dst[0]", "dst[1]", "dst[2]"};
    Range r[6];
    for (int i = 0; i < 6; ++i) {
        if (!p[i]) return fail(PW_ERR_INVALID_ARG, "%s is NULL", names[i]);
        if (reinterpret_cast<uintptr_t>(p[i]) % 16) return fail(PW_ERR_INVALID_ARG, "%s is not 16-byte aligned", names[i]);
        r[i] = Range{names[i], reinterpret_cast<uintptr_t>(p[i]), reinterpret_cast<uintptr_t>(p[i]) + uintptr_t(nbytes)};
    }
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j)
            if (overlap(r[i], r[j])) return fail(PW_ERR_INVALID_ARG, "%s and %s overlap", names[i], names[j]);
    int dev = 0;
    PW_TRY(current_device(&dev));
    for (int i = 0; i < 6; ++i) PW_TRY(check_on_device(names[i], p[i], dev));
    return launch_copy3(src, dst, nbytes, static_cast<hipStream_t>(hip_stream));
}

pw_status pw_stream_probe(int32_t mode, int32_t loads_per_lane, int32_t flags, const void *src, void *dst,
                          int64_t nbytes, int32_t blocks, void *hip_stream) {
    g_err[0] = 0;
    if (mode < 0 || mode > 2) return fail(PW_ERR_INVALID_ARG, "mode %d (0 copy, 1 read, 2 write)", mode);
    if (loads_per_lane != 1 && loads_per_lane != 2 && loads_per_lane != 4 && loads_per_lane != 8)
        return fail(PW_ERR_INVALID_ARG, "loads_per_lane %d (1, 2, 4 or 8)", loads_per_lane);
    if (flags & ~3) return fail(PW_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (blocks < 1 || blocks > (1 << 20)) return fail(PW_ERR_INVALID_ARG, "blocks %d out of 1..1048576", blocks);
    if (nbytes <= 0 || nbytes % 16) return fail(PW_ERR_INVALID_ARG, "nbytes must be a positive multiple of 16");
    const bool use_src = mode != 2;
    if ((use_src && !src) || !dst) return fail(PW_ERR_INVALID_ARG, "NULL pointer");
    if ((reinterpret_cast<uintptr_t>(use_src ? src : nullptr) | reinterpret_cast<uintptr_t>(dst)) % 16)
        return fail(PW_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    const int64_t dbytes = mode == 1 ? 4096 : nbytes;
    if (use_src) {
        const Range a{"src", reinterpret_cast<uintptr_t>(src), reinterpret_cast<uintptr_t>(src) + uintptr_t(nbytes)};
        const Range b{"dst", reinterpret_cast<uintptr_t>(dst), reinterpret_cast<uintptr_t>(dst) + uintptr_t(dbytes)};
        if (overlap(a, b)) return fail(PW_ERR_INVALID_ARG, "src and dst overlap");
    }
    int dev = 0;
    PW_TRY(current_device(&dev));
    if (use_src) PW_TRY(check_on_device("src", src, dev));
    PW_TRY(check_on_device("dst", dst, dev));
    return launch_probe(mode, loads_per_lane, flags, src, dst, nbytes, blocks, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
