// The fit kernels for a uniform field with FP32 stepping on an FP64 anchor (mixed precision).
#include "kf_fit_kernels.hpp"

namespace kffit {
hipError_t launch_fwd_uniform_mixed(KF_FWD_ARGS) {
    return launch_fwd<float, FIELD_UNIFORM>(a, sched, block, waves_per_cu, occ, split, storef, twof, curved, stream);
}
}  // namespace kffit
