// Forward kernel instantiations for FP32 storage with rows shared through LDS
// (see strip_march_lds in pw_stencil.h); the shapes are those
// shared_tile_supported accepts.
#include "pw_forward_impl.h"

namespace pw {

pw_status launch_forward_lds_f32(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    if (cfg.px == 4 && cfg.ry == 1) return fwd::launch_lds_t<float, 4, 1>(g, cfg, s);
    if (cfg.px == 4 && cfg.ry == 2) return fwd::launch_lds_t<float, 4, 2>(g, cfg, s);
    if (cfg.px == 4 && cfg.ry == 4) return fwd::launch_lds_t<float, 4, 4>(g, cfg, s);
    return fail(PW_ERR_UNSUPPORTED, "shared-row tile cols=%d rows=%d not instantiated", cfg.px, cfg.ry);
}

}  // namespace pw
