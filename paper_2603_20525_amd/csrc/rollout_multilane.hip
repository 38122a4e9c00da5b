// Two- and four-lane instantiations of the rollout kernels (see
// rollout_kernels.h).
#include "rollout_kernels.h"

namespace plan {

hipError_t launch_rollout_multi(const RolloutArgs &a, int lanes, int block, bool chunk,
                                hipStream_t s) {
    if (lanes == 2) return launch_rollout_lanes<2>(a, block, chunk, s);
    if (lanes == 4) return launch_rollout_lanes<4>(a, block, chunk, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sampled_multi(const RolloutArgs &a, int lanes, int block, hipStream_t s) {
    if (lanes == 2) return launch_sampled_lanes<2>(a, block, s);
    if (lanes == 4) return launch_sampled_lanes<4>(a, block, s);
    return hipErrorInvalidValue;
}

hipError_t launch_ckpt_multi(const RolloutArgs &a, int lanes, int block, hipStream_t s) {
    if (lanes == 2) return launch_ckpt_lanes<2>(a, block, s);
    if (lanes == 4) return launch_ckpt_lanes<4>(a, block, s);
    return hipErrorInvalidValue;
}

hipError_t launch_argmin_multi(const RolloutArgs &a, int lanes, int block, bool sampled,
                               hipStream_t s) {
    if (lanes == 2) return launch_argmin_lanes<2>(a, block, sampled, s);
    if (lanes == 4) return launch_argmin_lanes<4>(a, block, sampled, s);
    return hipErrorInvalidValue;
}

hipError_t launch_slots_multi(const RolloutArgs *slots, const TickTable &t, int *bad,
                              SelectOut *ring, uint32_t seq, bool s1, int lanes, int block,
                              hipStream_t s) {
    if (lanes == 2) return launch_slots_lanes<2>(slots, t, bad, ring, seq, s1, block, s);
    if (lanes == 4) return launch_slots_lanes<4>(slots, t, bad, ring, seq, s1, block, s);
    return hipErrorInvalidValue;
}

}  // namespace plan
