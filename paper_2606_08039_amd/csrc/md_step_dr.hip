// md_step_dr.hip -- instantiation of the persistent step kernel
// (md_step_kernel.h) with domain randomisation (per-drone constants, motor
// bias and lag, action and sensor latency, sensor noise and bias), with or
// without wind.
#include "md_step_kernel.h"

namespace md {

hipError_t launch_step_dr(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                          int n_bins, int slots, hipStream_t stream) {
    return launch_step_t<2>(a, mask, act, cfg, n_bins, slots, stream);
}

}  // namespace md
