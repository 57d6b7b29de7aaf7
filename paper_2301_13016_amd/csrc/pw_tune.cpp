// Autotuner for single-grid launches and its process-wide cache.
//
// The launch shape (columns per lane, rows per strip, z-chunks, wavefronts
// per workgroup) changes only speed, never results.  pw_tune times candidate
// shapes on scratch grids and keeps the fastest per kernel kind, dtype and
// shape class (the power-of-two ceilings of nx, ny, nz); pw_advect and
// pw_advect_adjoint use it when called without a tile.  The vertical cut is
// stored as a number of z-chunks, so one entry serves every nz of its class.
// With PWADV_TUNE_CACHE set, the table is read from that file on first use
// and rewritten after every pw_tune (one entry per line, plain text).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pw_internal.h"

namespace pw {
namespace {

int ceil_log2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

using Key = std::tuple<int, int, int, int, int>;   // kind, dtype, log2 nx, ny, nz
struct Entry {
    int px, ry, nzc, wpb;
};

std::mutex g_mu;
std::map<Key, Entry> g_table;
bool g_loaded = false;

Key make_key(TuneKind kind, const pw_grid *g, pw_dtype dt) {
    return Key(static_cast<int>(kind), static_cast<int>(dt), ceil_log2(g->nx), ceil_log2(g->ny), ceil_log2(g->nz));
}

const char *cache_path() {
    const char *p = std::getenv("PWADV_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// Called with g_mu held.
void load_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;   // a missing cache is an empty one
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        int kind, dt, lx, ly, lz, px, ry, nzc, wpb;
        if (std::sscanf(line, "pwadv-tune-v1 %d %d %d %d %d %d %d %d %d", &kind, &dt, &lx, &ly, &lz, &px, &ry, &nzc,
                        &wpb) == 9 &&
            nzc >= 1 && wpb >= 1 && wpb <= 8 && px >= 1 && ry >= 1)
            g_table[Key(kind, dt, lx, ly, lz)] = Entry{px, ry, nzc, wpb};
        // anything else (corrupt or foreign lines) is ignored
    }
    std::fclose(f);
}

void save_locked() {
    const char *path = cache_path();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto &kv : g_table) {
        int kind, dt, lx, ly, lz;
        std::tie(kind, dt, lx, ly, lz) = kv.first;
        std::fprintf(f, "pwadv-tune-v1 %d %d %d %d %d %d %d %d %d\n", kind, dt, lx, ly, lz, kv.second.px, kv.second.ry,
                     kv.second.nzc, kv.second.wpb);
    }
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

TileCfg entry_to_cfg(const Entry &e, int64_t zextent) {
    TileCfg c;
    c.px = e.px;
    c.ry = e.ry;
    c.wpb = e.wpb;
    c.zlen = static_cast<int>((zextent + e.nzc - 1) / e.nzc);
    if (c.zlen < 1) c.zlen = 1;
    return c;
}

// Timing helper: mean milliseconds of `reps` launches after one warm-up.
template <typename F> float time_ms(F launch, hipStream_t s, int reps, pw_status *st) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.f;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.f;
    }
    *st = launch();
    float ms = -1.f;
    if (*st == PW_OK && hipEventRecord(a, s) == hipSuccess) {
        for (int i = 0; i < reps && *st == PW_OK; ++i) *st = launch();
        if (*st == PW_OK && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
            hipEventElapsedTime(&ms, a, b) == hipSuccess)
            ms /= reps;
        else
            ms = -1.f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc(&p, n); }
};

}  // namespace

bool lookup_tuned(TuneKind kind, const pw_grid *grid, pw_dtype dt, TileCfg *cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_table.find(make_key(kind, grid, dt));
    if (it == g_table.end()) return false;
    const int64_t zext = kind == TuneKind::Adjoint ? grid->nz + 2 * grid->halo : grid->nz;
    *cfg = entry_to_cfg(it->second, zext);
    if (kind == TuneKind::Forward ? !tile_supported(*cfg, dt) : !adjoint_tile_supported(*cfg)) return false;
    return true;
}

void store_tuned(TuneKind kind, const pw_grid *grid, pw_dtype dt, const TileCfg &cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    const int64_t zext = kind == TuneKind::Adjoint ? grid->nz + 2 * grid->halo : grid->nz;
    Entry e{cfg.px, cfg.ry, static_cast<int>((zext + cfg.zlen - 1) / cfg.zlen), cfg.wpb};
    g_table[make_key(kind, grid, dt)] = e;
    save_locked();
}

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_tune(const pw_grid *grid, pw_dtype dtype, int32_t flags, pw_tile *fwd_best, pw_tile *adj_best) {
    if (!grid) return fail(PW_ERR_INVALID_ARG, "grid is NULL");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || grid->halo < 1 || grid->nx > (1 << 24) ||
        grid->ny > (1 << 24) || grid->nz > (1 << 24) || grid->halo > 1024)
        return fail(PW_ERR_INVALID_ARG, "bad grid extent");
    int64_t es = 0;
    switch (dtype) {
        case PW_F32: es = 4; break;
        case PW_F64: es = 8; break;
        case PW_BF16: case PW_F16: es = 2; break;
        default: return fail(PW_ERR_INVALID_ARG, "unknown dtype %d", static_cast<int>(dtype));
    }
    if (flags & ~(PW_TUNE_FORWARD | PW_TUNE_ADJOINT)) return fail(PW_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (flags == 0) flags = PW_TUNE_FORWARD | PW_TUNE_ADJOINT;
    const bool do_adj = (flags & PW_TUNE_ADJOINT) && (dtype == PW_F32 || dtype == PW_F64);
    const bool do_fwd = flags & PW_TUNE_FORWARD;
    const int64_t cs = dtype == PW_F64 ? 8 : 4;
    const int64_t px = grid->nx + 2 * grid->halo, py = grid->ny + 2 * grid->halo, pz = grid->nz + 2 * grid->halo;
    const int64_t npad = px * py * pz, nint = grid->nx * grid->ny * grid->nz;
    if (px * py * cs >= (int64_t(1) << 31)) return fail(PW_ERR_UNSUPPORTED, "a z-plane larger than 2 GiB");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return fail(PW_ERR_NO_DEVICE, "no usable HIP device");
    }

    DevBuf in, out, coef, grad;
    if (in.alloc(size_t(3 * npad * es)) != hipSuccess || out.alloc(size_t(3 * nint * cs)) != hipSuccess ||
        coef.alloc(size_t(4 * grid->nz * cs)) != hipSuccess ||
        (do_adj && grad.alloc(size_t(3 * npad * cs)) != hipSuccess)) {
        (void)hipGetLastError();
        return fail(PW_ERR_ALLOC, "scratch allocation for tuning failed");
    }
    hipStream_t s;
    if (hipStreamCreate(&s) != hipSuccess) return hip_fail(hipGetLastError(), "hipStreamCreate");
    hipError_t me = hipMemsetAsync(in.p, 0, size_t(3 * npad * es), s);
    if (me == hipSuccess) me = hipMemsetAsync(coef.p, 0, size_t(4 * grid->nz * cs), s);
    if (me != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(me, "scratch clear");
    }

    char *ib = static_cast<char *>(in.p), *ob = static_cast<char *>(out.p), *cb = static_cast<char *>(coef.p);
    FwdArgs a;
    a.u = ib; a.v = ib + npad * es; a.w = ib + 2 * npad * es;
    a.su = ob; a.sv = ob + nint * cs; a.sw = ob + 2 * nint * cs;
    a.tzc1 = cb; a.tzc2 = cb + grid->nz * cs; a.tzd1 = cb + 2 * grid->nz * cs; a.tzd2 = cb + 3 * grid->nz * cs;
    a.tcx = a.tcy = 0.0025;
    a.nx = grid->nx; a.ny = grid->ny; a.nz = grid->nz; a.h = grid->halo;
    a.in_sy = px; a.in_sz = px * py; a.out_sy = grid->nx; a.out_sz = grid->nx * grid->ny;
    a.in_bytes = es;
    a.out_bytes = cs;

    pw_status st = PW_OK;
    const int reps = 3;
    if (do_fwd) {
        float best = -1.f;
        TileCfg bestc = default_forward_tile(a, dtype);
        for (int pxl : {1, 2, 4})
            for (int ry : {1, 2, 4})
                for (int nzc : {1, 2, 4, 8})
                    for (int wpb : {1, 4}) {
                        TileCfg c;
                        c.px = pxl;
                        c.ry = ry;
                        c.wpb = wpb;
                        c.zlen = static_cast<int>((grid->nz + nzc - 1) / nzc);
                        if (!tile_supported(c, dtype) || (nzc > 1 && c.zlen < 4)) continue;
                        pw_status ls = PW_OK;
                        const float ms = time_ms([&] { return launch_forward(a, dtype, c, s); }, s, reps, &ls);
                        if (ls != PW_OK) {
                            st = ls;
                            break;
                        }
                        if (ms > 0.f && (best < 0.f || ms < best)) {
                            best = ms;
                            bestc = c;
                        }
                    }
        if (st == PW_OK) {
            store_tuned(TuneKind::Forward, grid, dtype, bestc);
            if (fwd_best) *fwd_best = pw_tile{bestc.px, bestc.ry, bestc.zlen, bestc.wpb};
        }
    }
    if (st == PW_OK && do_adj) {
        AdjArgs g;
        g.u = a.u; g.v = a.v; g.w = a.w;
        g.gsu = a.su; g.gsv = a.sv; g.gsw = a.sw;
        char *gb = static_cast<char *>(grad.p);
        g.gu = gb; g.gv = gb + npad * cs; g.gw = gb + 2 * npad * cs;
        g.tzc1 = a.tzc1; g.tzc2 = a.tzc2; g.tzd1 = a.tzd1; g.tzd2 = a.tzd2;
        g.tcx = g.tcy = 0.0025;
        g.nx = a.nx; g.ny = a.ny; g.nz = a.nz; g.h = a.h;
        g.in_sy = a.in_sy; g.in_sz = a.in_sz; g.out_sy = a.out_sy; g.out_sz = a.out_sz;
        if (hipMemsetAsync(out.p, 0, size_t(3 * nint * cs), s) != hipSuccess) st = hip_fail(hipGetLastError(), "clear");
        float best = -1.f;
        TileCfg bestc = default_adjoint_tile(g, dtype);
        for (int ry : {1, 2, 4})
            for (int nzc : {1, 2, 4, 8})
                for (int wpb : {1, 4}) {
                    TileCfg c;
                    c.px = 1;
                    c.ry = ry;
                    c.wpb = wpb;
                    c.zlen = static_cast<int>((pz + nzc - 1) / nzc);
                    if (!adjoint_tile_supported(c) || (nzc > 1 && c.zlen < 4)) continue;
                    pw_status ls = PW_OK;
                    const float ms = time_ms([&] { return launch_adjoint(g, dtype, c, s); }, s, reps, &ls);
                    if (ls != PW_OK) {
                        st = ls;
                        break;
                    }
                    if (ms > 0.f && (best < 0.f || ms < best)) {
                        best = ms;
                        bestc = c;
                    }
                }
        if (st == PW_OK) {
            store_tuned(TuneKind::Adjoint, grid, dtype, bestc);
            if (adj_best) *adj_best = pw_tile{bestc.px, bestc.ry, bestc.zlen, bestc.wpb};
        }
    }
    const hipError_t se = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (st != PW_OK) return st;
    return hip_fail(se, "tuning run");
}

pw_status pw_tune_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    g_loaded = true;   // do not reload the file into the emptied table
    return PW_OK;
}

}  // extern "C"
