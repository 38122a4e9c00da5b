// Candidate rollout kernel for the single-rigid-body (SRB) off-road vehicle
// model, with the stage cost and the energy-stability-margin (ESM) soft
// constraint fused into the integration loop (arXiv 2603.20525, sections
// "Single Rigid Body Vehicle Dynamics Model", "Energy Stability Margin
// Constraint", "OCP Formulation", "Real-Time Implementation").
//
// Layout and mapping (gfx950, wave64):
//   * LANES consecutive lanes simulate one candidate. The four wheels
//     (fl, fr, rl, rr) are split over those lanes (4/LANES wheels per lane);
//     the chassis part of each step (attitude, right-hand side, ESM, cost,
//     Euler update) is evaluated redundantly and bit-identically by every lane
//     of the group, so no broadcast is needed. Wheel sums use DPP quad
//     permutations in the fixed order (w0 + w1) + (w2 + w3) for every LANES,
//     so results do not depend on the launch shape.
//   * Arithmetic is fixed by the source: the library is compiled without
//     floating-point contraction and every fused multiply-add is an explicit
//     fmaf, so each launch shape and the chunked form produce the same bits.
//   * The 13-component state lives in VGPRs for the whole horizon; HBM traffic
//     inside the loop is the per-interval control pair (coalesced over k in the
//     [N][2][K] layout) and the terrain gathers, which hit L1/L2.
//   * Terrain: one 64-byte record per heightmap cell holding the bilinear
//     coefficients of (h, f_x, f_y, cost); software interpolation in FP32
//     (three multiply-adds per channel) with clamp-to-edge.
#include <string.h>

#include "rollout_kernels.h"

namespace plan {
namespace {

// controls [N][2][K] from the generator: thread (k, b) draws intervals
// 4b .. 4b+3 of candidate k from one generator block.
__global__ __launch_bounds__(256) void sample_controls(const SampleArgs sa, int K, int N,
                                                       float *__restrict__ controls) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (k >= K) return;
    const PhiloxBlock blk = sample_block(sa, k, b);
    const int n_end = min(4 * b + 4, N);
    for (int n = 4 * b; n < n_end; ++n) {
        float u0, u1;
        draw_controls(sa, block_word(blk, n & 3), k, n, u0, u1);
        controls[(2 * (size_t)n) * K + k] = u0;
        controls[(2 * (size_t)n + 1) * K + k] = u1;
    }
}

__global__ __launch_bounds__(256) void init_state(const RolloutArgs a) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= a.K) return;
#pragma unroll
    for (int q = 0; q < 13; ++q) a.state[(size_t)q * a.K + k] = a.s0[q];
    a.cost[k] = 0.0f;
}

}  // namespace

// Public dispatch: one lane here (or, with one_wave, in
// rollout_onelane_1wave.hip), two and four lanes in rollout_multilane.hip.
hipError_t launch_rollout(const RolloutArgs &a, int lanes, int block, bool chunk,
                          hipStream_t s, bool one_wave) {
    if (lanes != 1) return launch_rollout_multi(a, lanes, block, chunk, s);
    return one_wave ? launch_rollout_1wave(a, block, chunk, s)
                    : launch_rollout_lanes<1>(a, block, chunk, s);
}

hipError_t launch_rollout_sampled(const RolloutArgs &a, int lanes, int block, hipStream_t s,
                                  bool one_wave) {
    if (lanes != 1) return launch_sampled_multi(a, lanes, block, s);
    return one_wave ? launch_sampled_1wave(a, block, s) : launch_sampled_lanes<1>(a, block, s);
}

hipError_t launch_rollout_ckpt(const RolloutArgs &a, int lanes, int block, hipStream_t s) {
    return lanes == 1 ? launch_ckpt_lanes<1>(a, block, s) : launch_ckpt_multi(a, lanes, block, s);
}

hipError_t launch_rollout_argmin(const RolloutArgs &a, int lanes, int block, bool sampled,
                                 hipStream_t s, bool one_wave) {
    if (lanes != 1) return launch_argmin_multi(a, lanes, block, sampled, s);
    return one_wave ? launch_argmin_1wave(a, block, sampled, s)
                    : launch_argmin_lanes<1>(a, block, sampled, s);
}

int balanced_split(long long K, int simds) {
    const long long round = 64ll * simds;  // candidates of one wave per SIMD
    const long long R = K / round, rem = K - R * round;
    if (R < 1 || R > 3 || rem == 0 || 4 * rem > round) return 0;
    return (int)(R * round / 64);
}

hipError_t launch_rollout_balanced(const RolloutArgs &a, int split, bool sampled, bool fused,
                                   hipStream_t s) {
    const long long tail = (long long)a.K - 64ll * split;
    if (split < 1 || tail < 1) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(split + (tail * 4 + 63) / 64);
#define PLAN_LAUNCH(SMP, FU)                                                                    \
    if (sampled == SMP && fused == FU) {                                                        \
        hipLaunchKernelGGL((rollout_balanced<64, SMP, FU, false, false>), dim3(grid), dim3(64),  \
                           0, s, a, split);                                                     \
        return hipGetLastError();                                                               \
    }
    PLAN_LAUNCH(false, false)
    PLAN_LAUNCH(true, false)
    PLAN_LAUNCH(false, true)
    PLAN_LAUNCH(true, true)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_rollout_slots(const RolloutArgs *slots, const TickTable &t, int *bad,
                                SelectOut *ring, uint32_t seq, bool s1, int lanes, int block,
                                hipStream_t s) {
    if (t.count < 1) return hipSuccess;
    return lanes == 1 ? launch_slots_lanes<1>(slots, t, bad, ring, seq, s1, block, s)
                      : launch_slots_multi(slots, t, bad, ring, seq, s1, lanes, block, s);
}

hipError_t launch_sample_controls(const SampleArgs &sa, int K, int N, float *controls,
                                  hipStream_t s) {
    const dim3 grid((unsigned)((K + 255) / 256), (unsigned)((N + 3) / 4));
    hipLaunchKernelGGL(sample_controls, grid, dim3(256), 0, s, sa, K, N, controls);
    return hipGetLastError();
}

hipError_t launch_init_state(const float *s0, float *state, float *cost, int K, hipStream_t s) {
    RolloutArgs a;
    memset(&a, 0, sizeof a);
    for (int q = 0; q < 13; ++q) a.s0[q] = s0[q];
    a.state = state;
    a.cost = cost;
    a.K = K;
    hipLaunchKernelGGL(init_state, dim3((K + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace plan
