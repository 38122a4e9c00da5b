// One-lane instantiations of the rollout kernels (see rollout_kernels.h) for
// launches of at most one wave per SIMD, built with the max-ILP instruction
// scheduler: a wave that has its SIMD to itself has nothing to hide its
// per-step dependency chain behind, and the ILP schedule shortens that chain
// (2.6-4 % on the stress workload's 65 536 candidates, one wave per SIMD),
// while with three or four one-lane waves per SIMD (the paper's 204 288
// candidates) it is 2.6 % slower than the default schedule of rollout.hip.
// The forward-Euler kernels of one substep per interval with materialised
// controls run from rollout_onelane_ahead.hip instead.
#define PLAN_ONE_WAVE_PER_SIMD 1
#include "rollout_kernels.h"

namespace plan {

hipError_t launch_rollout_ilp1(const RolloutArgs &a, int block, bool chunk, hipStream_t s) {
    return launch_rollout_lanes<1>(a, block, chunk, s);
}

hipError_t launch_sampled_ilp1(const RolloutArgs &a, int block, hipStream_t s) {
    return launch_sampled_lanes<1>(a, block, s);
}

hipError_t launch_argmin_ilp1(const RolloutArgs &a, int block, bool sampled, hipStream_t s) {
    return launch_argmin_lanes<1>(a, block, sampled, s);
}

}  // namespace plan
