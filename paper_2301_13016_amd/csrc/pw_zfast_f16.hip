// z-fastest forward kernel instantiated for FP16 storage.
#include "pw_zfast_impl.h"

namespace pw {

pw_status launch_zfast_f16(const FwdArgs &a, const TileCfg &cfg, hipStream_t s) { return zf::launch_dt<_Float16>(a, cfg, s); }

}  // namespace pw
