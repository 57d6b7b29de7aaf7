// Internal declarations shared by the host API and the kernel translation units
// of libpwadv.  Not installed; the public interface is include/pwadv.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pwadv.h"

namespace pw {

// Launch shape of the forward / adjoint stencil kernels.
//   px     consecutive x columns per lane (forward: 1, 2, 4, 8; adjoint: 1; tangent: 1, 2)
//   ry     rows (y) per wavefront strip, a compile-time instantiation
//   zlen   z-levels per work item (the vertical march length; the grid is cut
//          into ceil(nz / zlen) independent chunks, each re-reading one plane
//          above and below)
//   wpb    wavefronts per workgroup (stacked in y), 1..8
//   depth  planes in flight ahead of the level being computed (forward: 1, 2;
//          the other kernels: 1)
struct TileCfg {
    int px = 1;
    int ry = 2;
    int zlen = 16;
    int wpb = 4;
    int depth = 1;
    int share = 0;   // pw_tile.share_rows
};
inline pw_tile to_tile(const TileCfg &c) { return pw_tile{c.px, c.ry, c.zlen, c.wpb, c.depth, c.share}; }
// A public launch shape as the kernels take it (prefetch 0 means 1).
inline TileCfg to_cfg(const pw_tile &t) {
    TileCfg c;
    c.px = t.cols_per_lane;
    c.ry = t.rows_per_strip;
    c.zlen = t.zlen;
    c.wpb = t.waves_per_group;
    c.depth = t.prefetch == 0 ? 1 : t.prefetch;
    c.share = t.share_rows;
    return c;
}

// Operands of one forward launch, already validated.  Strides are in elements.
struct FwdArgs {
    const void *u, *v, *w;
    void *su, *sv, *sw;
    const void *tzc1, *tzc2, *tzd1, *tzd2;
    double tcx, tcy;
    int64_t nx, ny, nz;
    int32_t h;
    int64_t in_sy, in_sz, out_sy, out_sz;
    int64_t in_bytes = 4, out_bytes = 4;   // element sizes of inputs / outputs
    // fused epilogue: out = c + alpha * F (epilogue == false: out = F)
    bool epilogue = false;
    const void *cu = nullptr, *cv = nullptr, *cw = nullptr;
    double alpha = 1.0;
    // boundary rules applied by addressing: the read remapping per axis
    // (KEEP, PERIODIC, or COPY = nearest interior cell) and the value rules
    // (byte d = axis x, y, z; 2 bits per field f = u, v, w at bit 2f:
    // 1 negate, 2 zero)
    int32_t bcx = PW_HALO_KEEP, bcy = PW_HALO_KEEP, bcz = PW_HALO_KEEP;
    uint32_t bcv = 0;
};

struct AdjArgs {
    const void *u, *v, *w;
    const void *gsu, *gsv, *gsw;
    void *gu, *gv, *gw;
    const void *tzc1, *tzc2, *tzd1, *tzd2;
    double tcx, tcy;
    int64_t nx, ny, nz;
    int32_t h;
    int64_t in_sy, in_sz, out_sy, out_sz;
};

// Operands of one tangent launch: the forward's (outputs tu, tv, tw in su, sv,
// sw) plus the direction, laid out like u, v, w.
struct TanArgs {
    FwdArgs f;
    const void *du, *dv, *dw;
};


// Operands of one halo fill (validated): up to kMaxHaloFields distinct
// padded arrays of element size es sharing one layout, with per-field x, y, z
// rules (pw_halo_mode).
constexpr int kMaxHaloFields = 8;
struct HaloArgs {
    void *f[kMaxHaloFields];
    int32_t mode[kMaxHaloFields][3];
    int32_t nf, es;
    int64_t nx, ny, nz;
    int32_t h;
    int64_t sy, sz;
};

// Columns of gradient produced by one adjoint wavefront: 64 lanes load 64
// consecutive padded columns and the 62 inner lanes own an output each.
constexpr int kWaveCols = 62;

bool tile_supported(const TileCfg &c, pw_dtype dt);
bool adjoint_tile_supported(const TileCfg &c);
TileCfg default_forward_tile(const FwdArgs &a, pw_dtype dt);
TileCfg default_adjoint_tile(const AdjArgs &a, pw_dtype dt);
bool tangent_tile_supported(const TileCfg &c, pw_dtype dt);
TileCfg default_tangent_tile(const TanArgs &a, pw_dtype dt);

pw_status launch_forward(const FwdArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s);
// per storage type (pw_forward_f32.hip, ...); launch_forward dispatches to these
pw_status launch_forward_f32(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_forward_f64(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_forward_bf16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_forward_f16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
// the same with a shared-row tile (cfg.share != 0), pw_forward_lds_{f32,...}.hip
pw_status launch_forward_lds_f32(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_forward_lds_f64(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_forward_lds_bf16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_forward_lds_f16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_adjoint(const AdjArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s);
// The adjoint march computing the wind gradients (grads), the per-strip
// coefficient partials (partials != NULL: [6][nz][adjoint_strips(g, cfg.ry)]
// doubles), or both in one pass; the coefficient fields of `a` are only read
// for the gradients.
pw_status launch_adjoint_mode(const AdjArgs &a, pw_dtype dt, const TileCfg &cfg, bool grads, double *partials,
                              hipStream_t s);
int64_t adjoint_strips(const pw_grid &g, int ry);
pw_status launch_tangent(const TanArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s);
int64_t coeff_grad_workspace_bytes(const pw_grid &g, pw_dtype dt);
// Passes 2 and 3 of the coefficient gradients: grad (6*nz + 2 doubles) from
// the partials of nstrips strips.
pw_status launch_coeff_grad_reduce(const double *partials, int64_t nstrips, double *grad, int64_t nz,
                                   hipStream_t s);
// Size of the library's own coefficient-gradient scratch, and its address on
// the current device (looked up once per device, no allocation).
constexpr int64_t kCoeffGradScratchBytes = PW_COEFF_GRAD_STATIC_MAX_BYTES;
pw_status coeff_grad_scratch(void **ptr);
pw_status launch_halo(const HaloArgs &a, hipStream_t s);
pw_status launch_halo_fold(const HaloArgs &a, hipStream_t s);   // es 4 or 8
// n elements of type dt set to seeded pseudo-random values uniform in
// [lo, hi): the autotuner's timing inputs (pw_tune_data.hip).
hipError_t fill_tuning_data(void *p, int64_t n, pw_dtype dt, uint32_t seed, float lo, float hi, hipStream_t s);
// z-fastest forward (pw_zfast.hip): FwdArgs carry the column stride in
// in_sy / out_sy and the x-plane stride in in_sz / out_sz; tile px = levels
// per lane, ry = y-rows per strip, zlen = x-columns per work item.
bool zfast_tile_supported(const TileCfg &c, pw_dtype dt);
TileCfg default_zfast_tile(const FwdArgs &a, pw_dtype dt);
pw_status launch_zfast(const FwdArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s);
// per storage type (pw_zfast_f32.hip, ...); launch_zfast dispatches to these
pw_status launch_zfast_f32(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_zfast_f64(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_zfast_bf16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_zfast_f16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s);
pw_status launch_copy(const void *src, void *dst, int64_t nbytes, hipStream_t s);
pw_status launch_probe(int mode, int loads, int flags, const void *src, void *dst, int64_t nbytes, int blocks,
                       hipStream_t s);
pw_status launch_copy3(const void *const *src, void *const *dst, int64_t nbytes, hipStream_t s);

// Host-side validation shared by pw_advect and the batched form (pw_api.cpp).
// validate_forward checks everything that needs no HIP call and fills the
// launch operands; check_forward_on_device then checks the device pointers.
pw_status validate_forward(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                           const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                           void *su, void *sv, void *sw, FwdArgs *out);
pw_status check_forward_on_device(const FwdArgs &a);
// Byte ranges [lo, hi) of the three inputs and three outputs of a launch.
void forward_ranges(const FwdArgs &a, uintptr_t (*in)[2], uintptr_t (*out)[2]);

// Autotune cache (pw_tune.cpp): best launch shape per kernel kind, dtype and
// shape class, filled by pw_tune and consulted when no tile is given.
enum class TuneKind { Forward = 0, Adjoint = 1, Tangent = 2, Zfast = 3 };
// PWADV_TILE: a forward launch shape for calls that give none (an override
// for experiments), the pw_tile fields in order separated by 'x' or ','; at
// least cols_per_lane, rows_per_strip and zlen (waves_per_group 4, prefetch 1
// and share_rows 0 when left out).  Read on every call.  Returns 0 when unset
// or empty, 1 with the shape, -1 when malformed.
int env_forward_tile(pw_tile *t);
bool lookup_tuned(TuneKind kind, const pw_grid *grid, pw_dtype dt, TileCfg *cfg);
void store_tuned(TuneKind kind, const pw_grid *grid, pw_dtype dt, const TileCfg &cfg);

// Error plumbing (pw_api.cpp).
pw_status fail(pw_status st, const char *fmt, ...);
pw_status hip_fail(hipError_t e, const char *what);
// Host-side logging (environment PWADV_LOG): one line per launch on stderr.
void log_launch(const char *entry, const pw_grid *g, pw_dtype dt, const TileCfg *c, const char *how);

}  // namespace pw
