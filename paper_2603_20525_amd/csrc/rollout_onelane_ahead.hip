// One-lane forward-Euler kernels of one substep per interval (materialised
// controls; plain, chunked and with the fused argmin) for launches of at most
// one wave per SIMD: each node's terrain is requested a whole step ahead
// (euler_step_ahead in rollout_step.h). Built with the default instruction
// scheduler, which on the stress workload (65 536 candidates, one wave per
// SIMD) runs this form 1.7 % faster than the max-ILP schedule
// (193.4 against 196.7 us); the other one-lane kernels for such launches stay
// in rollout_onelane_ilp.hip.
#define PLAN_REQUEST_AHEAD 1
#include "rollout_kernels.h"

namespace plan {

namespace {

template <bool CM>
hipError_t launch_ahead_cm(const RolloutArgs &a, int block, bool chunk, bool fused,
                           hipStream_t s) {
    const unsigned grid = (unsigned)(((long long)a.K + block - 1) / block);
#define PLAN_LAUNCH(B)                                                                          \
    if (block == B) {                                                                           \
        if (fused)                                                                              \
            hipLaunchKernelGGL((rollout_srb<1, B, false, false, true, false, false, true, CM>),  \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        else if (chunk)                                                                         \
            hipLaunchKernelGGL((rollout_srb<1, B, true, false, false, false, false, true, CM>),  \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        else                                                                                    \
            hipLaunchKernelGGL((rollout_srb<1, B, false, false, false, false, false, true, CM>), \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        return hipGetLastError();                                                               \
    }
    PLAN_LAUNCH(64)
    PLAN_LAUNCH(256)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_rollout_ahead1(const RolloutArgs &a, int block, bool chunk, bool fused,
                                 hipStream_t s) {
    if (a.method != 0 || a.S != 1) return hipErrorInvalidValue;
    return a.has_costmap ? launch_ahead_cm<true>(a, block, chunk, fused, s)
                         : launch_ahead_cm<false>(a, block, chunk, fused, s);
}

}  // namespace plan
