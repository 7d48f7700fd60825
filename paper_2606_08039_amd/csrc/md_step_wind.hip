// md_step_wind.hip -- instantiation of the persistent step kernel
// (md_step_kernel.h) with wind and the nominal constants: the wind state and
// its Philox draws without the randomisation's per-drone registers.
#include "md_step_kernel.h"

namespace md {

hipError_t launch_step_wind(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                            int n_bins, int slots, hipStream_t stream) {
    return launch_step_t<1>(a, mask, act, cfg, n_bins, slots, stream);
}

}  // namespace md
