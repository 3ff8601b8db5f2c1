// The fit kernels for the solenoid field with FP64 stepping.
#include "kf_fit_kernels.hpp"

namespace kffit {
hipError_t launch_fwd_solenoid_fp64(KF_FWD_ARGS) {
    return launch_fwd<double, FIELD_SOLENOID>(a, sched, block, waves_per_cu, occ, split, storef, twof, curved, stream);
}
}  // namespace kffit
