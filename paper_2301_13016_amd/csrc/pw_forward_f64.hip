// Forward kernel instantiations for FP64 storage (see pw_forward_impl.h).
#include "pw_forward_impl.h"

namespace pw {

pw_status launch_forward_f64(const FwdArgs &g, const TileCfg &cfg, hipStream_t s) {
    return fwd::launch_fwd_dt<double>(g, cfg, s);
}

}  // namespace pw
