// z-fastest forward kernel instantiated for FP32 storage.
#include "pw_zfast_impl.h"

namespace pw {

pw_status launch_zfast_f32(const FwdArgs &a, const TileCfg &cfg, hipStream_t s) { return zf::launch_dt<float>(a, cfg, s); }

}  // namespace pw
