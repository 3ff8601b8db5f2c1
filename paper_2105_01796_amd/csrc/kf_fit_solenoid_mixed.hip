// The fit kernels for the solenoid field with FP32 stepping on an FP64 anchor (mixed precision).
#include "kf_fit_kernels.hpp"

namespace kffit {
hipError_t launch_fwd_solenoid_mixed(KF_FWD_ARGS) {
    return launch_fwd<float, FIELD_SOLENOID>(a, sched, block, waves_per_cu, occ, split, storef, twof, curved, stream);
}
}  // namespace kffit
