// z-fastest forward: launch-shape rules, default shape and dispatch to the
// per-storage-type translation units (the kernel is in pw_zfast_impl.h).
#include "pw_internal.h"

namespace pw {

bool zfast_tile_supported(const TileCfg &c, pw_dtype dt) {
    if (c.zlen < 1 || c.wpb < 1 || c.wpb > 8 || (c.depth != 1 && c.depth != 2) || c.share != 0) return false;
    const bool pz_ok = c.px == 1 || c.px == 2 || (c.px == 4 && dt != PW_F64);
    const bool ry_ok = c.ry == 1 || c.ry == 2 || (c.ry == 4 && c.px <= 2) || (c.ry == 8 && c.px == 1);
    return pz_ok && ry_ok;
}

TileCfg default_zfast_tile(const FwdArgs &a, pw_dtype dt) {
    // Measured on MI355X (512x512x64 and 256x256x128, FP32): one level per
    // lane up to 64 levels, two above (FP64: one); four-row strips; two
    // x-planes in flight; x-chunks for about 1024 wavefronts.
    TileCfg c;
    c.px = (a.nz > 64 && dt != PW_F64) ? 2 : 1;
    c.ry = 4;
    c.wpb = 4;
    c.depth = 2;
    const int64_t tiles = ((a.nz + 64 * c.px - 1) / (64 * c.px)) * ((a.ny + c.ry - 1) / c.ry);
    int64_t chunks = (1024 + tiles - 1) / tiles;
    if (chunks < 1) chunks = 1;
    int64_t xl = (a.nx + chunks - 1) / chunks;
    if (xl < 8) xl = 8;
    if (xl > a.nx) xl = a.nx;
    c.zlen = static_cast<int>(xl);
    return c;
}

pw_status launch_zfast(const FwdArgs &a, pw_dtype dt, const TileCfg &cfg, hipStream_t s) {
    if (!zfast_tile_supported(cfg, dt)) return fail(PW_ERR_INVALID_ARG, "unsupported z-fastest tile configuration");
    switch (dt) {
        case PW_F32: return launch_zfast_f32(a, cfg, s);
        case PW_F64: return launch_zfast_f64(a, cfg, s);
        case PW_BF16: return launch_zfast_bf16(a, cfg, s);
        case PW_F16: return launch_zfast_f16(a, cfg, s);
    }
    return fail(PW_ERR_UNSUPPORTED, "dtype %d", static_cast<int>(dt));
}

}  // namespace pw
