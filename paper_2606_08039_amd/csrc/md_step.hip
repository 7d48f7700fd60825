// md_step.hip -- instantiation of the persistent step kernel (md_step_kernel.h)
// with the nominal constants for every drone.
#include "md_step_kernel.h"

namespace md {

hipError_t launch_step(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                       int n_bins, int slots, hipStream_t stream) {
    return launch_step_t<0>(a, mask, act, cfg, n_bins, slots, stream);
}

}  // namespace md
