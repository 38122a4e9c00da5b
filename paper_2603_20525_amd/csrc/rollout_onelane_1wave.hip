// One-lane instantiations of the rollout kernels (see rollout_kernels.h) for
// launches of at most one wave per SIMD. Such a wave has its SIMD to itself,
// so registers are not needed for occupancy: these kernels carry no
// four-wave launch bound, and the forward-Euler ones of one substep per
// interval request each node's terrain a whole step ahead (euler_step_ahead),
// which holds two nodes' cell records in registers at once.
#define PLAN_ONE_WAVE_PER_SIMD 1
#define PLAN_REQUEST_AHEAD 1
#include "rollout_kernels.h"

namespace plan {

hipError_t launch_rollout_1wave(const RolloutArgs &a, int block, bool chunk, hipStream_t s) {
    return launch_rollout_lanes<1>(a, block, chunk, s);
}

hipError_t launch_sampled_1wave(const RolloutArgs &a, int block, hipStream_t s) {
    return launch_sampled_lanes<1>(a, block, s);
}

hipError_t launch_argmin_1wave(const RolloutArgs &a, int block, bool sampled, hipStream_t s) {
    return launch_argmin_lanes<1>(a, block, sampled, s);
}

}  // namespace plan
