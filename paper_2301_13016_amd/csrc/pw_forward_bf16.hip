// Forward kernel instantiations for BF16 (uint16_t bit patterns) storage (see pw_forward_impl.h).
#include "pw_forward_impl.h"

namespace pw {

pw_status launch_forward_bf16(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    return fwd::launch_fwd_dt<uint16_t>(g, cfg, s);
}

}  // namespace pw
