// z-fastest forward kernel instantiated for BF16 storage.
#include "pw_zfast_impl.h"

namespace pw {

pw_status launch_zfast_bf16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s) { return zf::launch_dt<uint16_t>(a, cfg, s); }

}  // namespace pw
