// Rollout kernel templates (SRB model, stage cost, ESM constraint) and, per
// lane count, their launch dispatch. Three translation units instantiate
// them: rollout.hip (one lane per candidate), rollout_onelane_1wave.hip (one
// lane per candidate for launches of at most one wave per SIMD) and
// rollout_multilane.hip (two and four lanes per candidate). The arithmetic is
// the same in all, so results are identical for every launch shape.
#pragma once

#include "plan_internal.h"
#include "rollout_step.h"
#include "select_common.h"

namespace plan {
namespace {

// The kernels built with PLAN_REQUEST_AHEAD (rollout_onelane_1wave.hip: one
// lane, launches of at most one wave per SIMD) have registers to spare: their
// Euler kernels with one substep per interval request each node's terrain a
// whole step ahead (euler_step_ahead), which holds two nodes' cell
// coefficients in registers at once (190-260 VGPRs). The one-lane kernels
// for three or four waves per SIMD (the paper's solver shape) need the
// registers for occupancy; the two- and four-lane kernels measured no gain
// (a wave there gathers one or two wheels' cells and waits mostly on its
// own dependency chain).
#ifdef PLAN_REQUEST_AHEAD
constexpr bool REQUEST_AHEAD = true;
#else
constexpr bool REQUEST_AHEAD = false;
#endif

// One candidate k over control intervals [a.n0, a.n1), simulated by the
// LANES lanes of its group (this lane is number sub). CHUNK: start from and
// write back a.state / a.cost; otherwise start from a.s0 with zero cost and
// write a.cost / a.final_state. SAMPLED: draw the controls from a.smp (one
// generator block per four intervals, kept in registers) instead of reading
// a.controls. Lanes with store == false run a duplicate candidate only to
// keep their lane group complete.
template <int LANES, bool CHUNK, bool SAMPLED = false, bool RK4 = false, bool CKPT = false,
          bool S1 = false, bool CM = true>
__device__ __forceinline__ float simulate(const RolloutArgs &a, int k, int sub, bool store,
                                          const float *up) {
    constexpr int WPL = 4 / LANES;  // wheels per lane
    const size_t K = (size_t)a.K;

    float st0[13];
    float J;
    if constexpr (CHUNK) {
#pragma unroll
        for (int q = 0; q < 13; ++q) st0[q] = a.state[(size_t)q * K + k];
        J = a.cost[k];
    } else {
#pragma unroll
        for (int q = 0; q < 13; ++q) st0[q] = a.s0[q];
        J = 0.0f;
    }
    float (&st)[13] = st0;

    // materialised controls are read one interval ahead (the index is clamped
    // to [n0, n1)). The Euler step requests the next pair right after its
    // terrain gathers, so waiting for the texels does not wait for it and the
    // load stays in flight for the rest of the step; RK4 requests it at the
    // start of the interval.
    // up: this candidate's control column (interval n at up[2 n K], up[(2 n + 1) K])
    float nu0 = 0.0f, nu1 = 0.0f;
    // the pair requested during interval n: interval min(n + 1, n1 - 1)
    const float *unext = up + 2 * (size_t)max(min(a.n0 + 1, a.n1 - 1), 0) * K;
    if constexpr (!SAMPLED) {
        if (a.n0 < a.n1) {
            nu0 = up[(2 * (size_t)a.n0) * K];
            nu1 = up[(2 * (size_t)a.n0 + 1) * K];
        }
    }
    PhiloxBlock blk{};
    int blk_n = -1;

    Arm arms[WPL];
#pragma unroll
    for (int q = 0; q < WPL; ++q) arms[q] = arm(a, sub * WPL + q);

    // CKPT: ckpt[b] = state at interval min(b C, N), the 13 stores spread over
    // the lane group; a candidate past its goal exit keeps its frozen state
    int ckpt_done = 0;
    auto write_ckpt = [&](int b) {
        if (!store) return;
        float *c = a.ckpt + (size_t)b * 13 * K + k;
#pragma unroll
        for (int q = 0; q < 13; ++q)
            if ((q & (LANES - 1)) == sub) c[(size_t)q * K] = st[q];
    };
    if constexpr (CKPT) write_ckpt(0);

    // Euler with one substep per interval in a request-ahead build: the
    // terrain of each node is requested a step ahead. The loop
    // takes two intervals per trip so that the two nodes' requests alternate
    // between two register sets (P, Q) instead of being copied from one to
    // the other, which would wait for the loads in flight. A candidate at its
    // goal skips the step and its requests; it stays frozen, so it never uses
    // a set again.
    constexpr bool AHEAD = REQUEST_AHEAD && !RK4 && !CKPT && S1;
    if constexpr (AHEAD) {
        auto interval = [&](int n, const NodeRequest<LANES, CM> &cur,
                            NodeRequest<LANES, CM> &nxt) {
            float u0, u1;
            if constexpr (SAMPLED) {
                if ((n >> 2) != blk_n) {
                    blk_n = n >> 2;
                    blk = sample_block(a.smp, k, blk_n);
                }
                draw_controls(a.smp, block_word(blk, n & 3), k, n, u0, u1);
            } else {
                u0 = nu0;
                u1 = nu1;
            }
            const float dd = clampf_nan(u0, -a.drate_max, a.drate_max);
            const float ax = a.accel_max * clampf_nan(u1, -1.0f, 1.0f);
            // goal test at the node, written as in the other loop so that a
            // NaN position (never at the goal) keeps stepping there as here
            const float gdx = st[0] - a.goal_x, gdy = st[1] - a.goal_y;
            if (!(fmaf(gdx, gdx, gdy * gdy) <= a.goal_r2)) {
                if constexpr (SAMPLED) {
                    euler_step_ahead<LANES, CM>(a, arms, st, J, dd, ax, cur, nxt);
                } else {
                    euler_step_ahead<LANES, CM>(a, arms, st, J, dd, ax, cur, nxt, [&]() {
                        nu0 = unext[0];
                        nu1 = unext[K];
                    });
                }
            }
            if (n + 2 < a.n1) unext += 2 * K;
        };
        NodeRequest<LANES, CM> P, Q;
        request_node<LANES, CM>(a, arms, st[0], st[1], st[2], st[3], st[4], st[5], P);
        int n = a.n0;
        for (; n + 1 < a.n1; n += 2) {
            interval(n, P, Q);
            interval(n + 1, Q, P);
        }
        if (n < a.n1) interval(n, P, Q);
    } else {
    // uniform trip counts: a candidate that reaches the goal stays in the
    // loop frozen (its lanes skip the steps), so the loops carry no
    // per-lane exit or done-flag bookkeeping
    for (int n = a.n0; n < a.n1; ++n) {
        // zero-order hold: control n for the whole interval, restricted to the
        // admissible set (|delta_dot| <= limit, throttle in [-1, 1])
        float u0, u1;
        if constexpr (SAMPLED) {
            if ((n >> 2) != blk_n) {
                blk_n = n >> 2;
                blk = sample_block(a.smp, k, blk_n);
            }
            draw_controls(a.smp, block_word(blk, n & 3), k, n, u0, u1);
        } else {
            u0 = nu0;
            u1 = nu1;
            if constexpr (RK4) {
                if (n + 1 < a.n1) {
                    nu0 = up[(2 * (size_t)n + 2) * K];
                    nu1 = up[(2 * (size_t)n + 3) * K];
                }
            }
        }
        const float dd = clampf_nan(u0, -a.drate_max, a.drate_max);
        const float ax = a.accel_max * clampf_nan(u1, -1.0f, 1.0f);

        // S1: one Euler substep per interval, no substep loop
        const int S = S1 ? 1 : a.S;
        for (int s = 0; s < S; ++s) {
            // goal test at the Euler node, before the step; a candidate at
            // its goal is frozen, so the test stays true for it from then on
            {
                const float gdx = st[0] - a.goal_x, gdy = st[1] - a.goal_y;
                if (fmaf(gdx, gdx, gdy * gdy) <= a.goal_r2) continue;
            }
            if constexpr (RK4) {
                rk4_step<LANES, CM>(a, arms, st, J, dd, ax);
            } else if constexpr (SAMPLED) {
                euler_step<LANES, CM>(a, arms, st, J, dd, ax);
            } else {
                euler_step<LANES, CM>(a, arms, st, J, dd, ax, [&]() {
                    nu0 = unext[0];
                    nu1 = unext[K];
                });
            }
        }
        if (n + 2 < a.n1) unext += 2 * K;
        if constexpr (CKPT) {
            if ((n + 1) % a.ckpt_every == 0 && n + 1 < a.N) {
                ckpt_done = (n + 1) / a.ckpt_every;
                write_ckpt(ckpt_done);
            }
        }
    }
    }
    if constexpr (CKPT) {
        const int nseg = (a.N + a.ckpt_every - 1) / a.ckpt_every;
        for (int b = ckpt_done + 1; b <= nseg; ++b) write_ckpt(b);
    }

    if (a.finalize) {
        // terminal cost at the final (or goal-exit) state; a non-finite cost
        // or state scores +inf
        const float gdx = st[0] - a.goal_x, gdy = st[1] - a.goal_y;
        J = fmaf(a.w_g, sqrtf(fmaf(gdx, gdx, gdy * gdy)), J);
        bool fin = isfinite(J);
#pragma unroll
        for (int q = 0; q < 13; ++q) fin = fin && isfinite(st[q]);
        if (!fin) J = __builtin_inff();
    }

    if (store) {
        if (sub == 0) a.cost[k] = J;
        float *out = CHUNK ? a.state : a.final_state;
        if (out) {
            // spread the 13 stores over the lane group
#pragma unroll
            for (int q = 0; q < 13; ++q)
                if ((q & (LANES - 1)) == sub) out[(size_t)q * K + k] = st[q];
        }
    }
    return J;
}

// Fused argmin: every workgroup reduces its candidates' packed keys and
// folds the result into a.sel_key with an atomic minimum (order-independent,
// so the winner is the same as the separate selection kernel's); the last of
// the nblocks workgroups to arrive publishes (k*, J*) to a.sel_out and
// out_host, writes the plan and resets the key and the ticket for the next
// launch. bad (optional) is a flag to report in the result's status and
// clear.
template <int BLOCK, bool SAMPLED>
__device__ __forceinline__ void argmin_epilogue(const RolloutArgs &a, unsigned long long key,
                                                unsigned int nblocks, SelectOut *out_host,
                                                int *bad) {
    __shared__ unsigned long long red[BLOCK / 64];
    __shared__ int last_sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    key = wave_min(key);
    if (lane == 0) red[wv] = key;
    __syncthreads();
    if (tid == 0) {
        unsigned long long b = red[0];
#pragma unroll
        for (int q = 1; q < BLOCK / 64; ++q) b = red[q] < b ? red[q] : b;
        last_sh = fold_key_and_take_ticket(a.sel_key, a.sel_ticket, b, nblocks);
    }
    __syncthreads();
    if (!last_sh) return;
    if (tid == 0) {
        const unsigned long long m = take_key_and_reset(a.sel_key, a.sel_ticket);
        red[0] = m;
        const int32_t status = (bad && *bad) ? (int32_t)PLAN_EINVAL : 0;
        if (bad) *bad = 0;  // the slot's next request starts with a clear flag
        publish_result(a.sel_out, out_host, m, a.sel_seq, status);
    }
    __syncthreads();
    const unsigned long long m = red[0];
    const int kb = (m == ~0ull) ? -1 : (int)(unsigned int)(m & 0xffffffffu);
    write_plan<SAMPLED>(kb, a.N, a.K, a.controls, a.smp, a.drate_max, a.plan, tid, BLOCK);
}

// One-lane full-horizon launches with several Euler substeps per interval and
// no costmap (the paper's solver shape) are held to 128 VGPRs, four waves per
// SIMD, so its 204 288 candidates (3.1 waves per SIMD) run in one round
// instead of three full rounds and a tail: the materialised-control kernel
// fits in 126 registers, the in-kernel-sampled one spills 15-17 registers
// (its generator words, read once per interval) and is 4.7 % faster all the
// same (2.93 -> 2.79 ms per ordered plan).
// (The instantiation for launches of at most one wave per SIMD, built with
// PLAN_ONE_WAVE_PER_SIMD, has no use for the bound.)
#ifdef PLAN_ONE_WAVE_PER_SIMD
template <int LANES, bool CHUNK, bool RK4, bool CKPT, bool S1, bool CM>
constexpr bool ONE_LANE_4_WAVES = false;
#else
template <int LANES, bool CHUNK, bool RK4, bool CKPT, bool S1, bool CM>
constexpr bool ONE_LANE_4_WAVES = LANES == 1 && !CHUNK && !RK4 && !CKPT && !S1 && !CM;
#endif

template <int LANES, int BLOCK, bool CHUNK, bool SAMPLED = false, bool FUSED = false,
          bool RK4 = false, bool CKPT = false, bool S1 = false, bool CM = true>
__global__ __launch_bounds__(BLOCK, (ONE_LANE_4_WAVES<LANES, CHUNK, RK4, CKPT, S1, CM> ? 4 : 1))
void rollout_srb(const RolloutArgs a) {
    const int gtid = blockIdx.x * BLOCK + threadIdx.x;
    const int sub = gtid & (LANES - 1);
    int slot = gtid / LANES;
    const bool store = slot < a.K;
    // Lanes past K simulate the last candidate again so that every lane group
    // is complete for the DPP sums; they store nothing (and reach the fused
    // epilogue's barriers like every other lane).
    if (!store) slot = a.K - 1;
    int k = slot;
    const float *up = a.controls + slot;
    if constexpr (LANES == 1 && !CHUNK && !CKPT) {
        // ordered launches run one lane per candidate
        if (a.order) {
            // clamped so that a malformed order can only misassign, never
            // address outside the candidate arrays
            k = min(max(a.order[slot], 0), a.K - 1);
            up = a.controls_lane ? a.controls_lane + slot : a.controls + k;
        }
    }
    const float J = simulate<LANES, CHUNK, SAMPLED, RK4, CKPT, S1, CM>(a, k, sub, store, up);
    if constexpr (FUSED)
        argmin_epilogue<BLOCK, SAMPLED>(a, (store && sub == 0) ? cost_key(J, k) : ~0ull,
                                        gridDim.x, a.sel_out_host, nullptr);
}

// A one-lane full-horizon launch whose candidates fill R whole rounds of one
// wave per SIMD plus a small remainder (the paper's 204 288 candidates are
// 3.12 waves per SIMD): run one lane per candidate would give that remainder
// a fourth wave on a few SIMDs and make the whole launch wait for them.
// Here workgroups [0, split) run one lane per candidate on slots
// [0, split x BLOCK) and the rest run four lanes per candidate on the
// remaining slots, so the remainder's work (about half a one-lane wave per
// 16 candidates) spreads over four times as many SIMDs. Every candidate's
// arithmetic is the same at any lane count, so results equal the one-lane
// launch's bit for bit. Held to four waves per SIMD like the one-lane kernel
// of the same shape.
template <int BLOCK, bool SAMPLED, bool FUSED, bool S1, bool CM>
__global__ __launch_bounds__(BLOCK, 4) void rollout_balanced(const RolloutArgs a, int split) {
    const bool four = (int)blockIdx.x >= split;  // uniform over the workgroup
    int slot, sub;
    if (!four) {
        slot = (int)blockIdx.x * BLOCK + (int)threadIdx.x;
        sub = 0;
    } else {
        const int g = ((int)blockIdx.x - split) * BLOCK + (int)threadIdx.x;
        slot = split * BLOCK + (g >> 2);
        sub = g & 3;
    }
    const bool store = slot < a.K;
    if (!store) slot = a.K - 1;
    int k = slot;
    const float *up = a.controls + slot;
    if (a.order) {
        k = min(max(a.order[slot], 0), a.K - 1);
        up = a.controls_lane ? a.controls_lane + slot : a.controls + k;
    }
    float J;
    if (four)
        J = simulate<4, false, SAMPLED, false, false, S1, CM>(a, k, sub, store, up);
    else
        J = simulate<1, false, SAMPLED, false, false, S1, CM>(a, k, 0, store, up);
    if constexpr (FUSED)
        argmin_epilogue<BLOCK, SAMPLED>(a, (store && sub == 0) ? cost_key(J, k) : ~0ull,
                                        gridDim.x, a.sel_out_host, nullptr);
}

// Several independent plans in one launch (the serving loop's tick). Entry e
// of the table owns blocks [e.block_start, next block_start) and advances
// slot e.slot through intervals [e.n0, e.n1); every block belongs to exactly
// one slot, so the per-slot arguments are wave-uniform. An entry that ends
// its request's horizon also selects the request's plan: the entry's blocks
// run the fused argmin epilogue on the slot's own key and ticket, and the
// last of them writes the result to ring[slot] and the plan.
template <int LANES, int BLOCK, bool S1>
__global__ __launch_bounds__(BLOCK) void rollout_slots(const RolloutArgs *__restrict__ slots,
                                                       const TickTable t, int *bad,
                                                       SelectOut *ring, uint32_t seq) {
    int lo = 0, hi = t.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.e[mid].block_start <= (int)blockIdx.x)
            lo = mid;
        else
            hi = mid - 1;
    }
    const TickEntry te = t.e[lo];
    const int block_end = lo + 1 < t.count ? t.e[lo + 1].block_start : t.total_blocks;
    RolloutArgs a = slots[te.slot];
    a.n0 = te.n0;
    a.n1 = te.n1;
    a.finalize = te.finalize;
    a.sel_seq = seq;
    const int gtid = ((int)blockIdx.x - te.block_start) * BLOCK + threadIdx.x;
    const int sub = gtid & (LANES - 1);
    int k = gtid / LANES;
    const bool store = k < a.K;
    if (!store) k = a.K - 1;
    const float J = simulate<LANES, true, false, false, false, S1>(a, k, sub, store,
                                                                   a.controls + k);
    if (te.finalize)
        argmin_epilogue<BLOCK, false>(a, (store && sub == 0) ? cost_key(J, k) : ~0ull,
                                      (unsigned int)(block_end - te.block_start),
                                      ring + te.slot, bad + te.slot);
}

// Launch dispatch for one lane count L (block 64 or 256) and costmap flag CM
// (the context's a.has_costmap). Euler launches with one substep per interval
// (a.S == 1) use the S1 instantiations, which carry no substep loop.
template <int L, bool CM>
__forceinline__ hipError_t launch_rollout_cm(const RolloutArgs &a, int block, bool chunk,
                                             hipStream_t s) {
    const long long threads = (long long)a.K * L;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
#define PLAN_LAUNCH(B, C)                                                                       \
    if (block == B && chunk == C) {                                                             \
        if (a.method == 1)                                                                      \
            hipLaunchKernelGGL((rollout_srb<L, B, C, false, false, true, false, false, CM>),     \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        else if (a.S == 1)                                                                      \
            hipLaunchKernelGGL((rollout_srb<L, B, C, false, false, false, false, true, CM>),     \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        else                                                                                    \
            hipLaunchKernelGGL((rollout_srb<L, B, C, false, false, false, false, false, CM>),    \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        return hipGetLastError();                                                               \
    }
    PLAN_LAUNCH(64, false)
    PLAN_LAUNCH(256, false)
    PLAN_LAUNCH(64, true)
    PLAN_LAUNCH(256, true)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

template <int L>
__forceinline__ hipError_t launch_rollout_lanes(const RolloutArgs &a, int block, bool chunk,
                                                hipStream_t s) {
    return a.has_costmap ? launch_rollout_cm<L, true>(a, block, chunk, s)
                         : launch_rollout_cm<L, false>(a, block, chunk, s);
}

template <int L, bool CM>
__forceinline__ hipError_t launch_sampled_cm(const RolloutArgs &a, int block, hipStream_t s) {
    const long long threads = (long long)a.K * L;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
    if (block == 64)
        hipLaunchKernelGGL((rollout_srb<L, 64, false, true, false, false, false, false, CM>),
                           dim3(grid), dim3(64), 0, s, a);
    else if (block == 256)
        hipLaunchKernelGGL((rollout_srb<L, 256, false, true, false, false, false, false, CM>),
                           dim3(grid), dim3(256), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int L>
__forceinline__ hipError_t launch_sampled_lanes(const RolloutArgs &a, int block, hipStream_t s) {
    return a.has_costmap ? launch_sampled_cm<L, true>(a, block, s)
                         : launch_sampled_cm<L, false>(a, block, s);
}

template <int L>
__forceinline__ hipError_t launch_ckpt_lanes(const RolloutArgs &a, int block, hipStream_t s) {
    const long long threads = (long long)a.K * L;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
#define PLAN_LAUNCH(B)                                                                          \
    if (block == B) {                                                                           \
        if (a.S == 1)                                                                           \
            hipLaunchKernelGGL((rollout_srb<L, B, false, false, false, false, true, true>),      \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        else                                                                                    \
            hipLaunchKernelGGL((rollout_srb<L, B, false, false, false, false, true>),            \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        return hipGetLastError();                                                               \
    }
    PLAN_LAUNCH(64)
    PLAN_LAUNCH(256)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

template <int L, bool CM>
__forceinline__ hipError_t launch_argmin_cm(const RolloutArgs &a, int block, bool sampled,
                                            hipStream_t s) {
    const long long threads = (long long)a.K * L;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
#define PLAN_LAUNCH(B)                                                                          \
    if (block == B) {                                                                           \
        if (sampled)                                                                            \
            hipLaunchKernelGGL((rollout_srb<L, B, false, true, true, false, false, false, CM>),  \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        else if (a.S == 1)                                                                      \
            hipLaunchKernelGGL((rollout_srb<L, B, false, false, true, false, false, true, CM>),  \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        else                                                                                    \
            hipLaunchKernelGGL((rollout_srb<L, B, false, false, true, false, false, false, CM>), \
                               dim3(grid), dim3(B), 0, s, a);                                   \
        return hipGetLastError();                                                               \
    }
    PLAN_LAUNCH(64)
    PLAN_LAUNCH(256)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

template <int L>
__forceinline__ hipError_t launch_argmin_lanes(const RolloutArgs &a, int block, bool sampled,
                                               hipStream_t s) {
    return a.has_costmap ? launch_argmin_cm<L, true>(a, block, sampled, s)
                         : launch_argmin_cm<L, false>(a, block, sampled, s);
}

// s1: every slot of the tick integrates with one substep per interval.
template <int L>
__forceinline__ hipError_t launch_slots_lanes(const RolloutArgs *slots, const TickTable &t,
                                              int *bad, SelectOut *ring, uint32_t seq, bool s1,
                                              int block, hipStream_t s) {
    const unsigned grid = (unsigned)t.total_blocks;
#define PLAN_LAUNCH(B)                                                                          \
    if (block == B) {                                                                           \
        if (s1)                                                                                 \
            hipLaunchKernelGGL((rollout_slots<L, B, true>), dim3(grid), dim3(B), 0, s, slots,    \
                               t, bad, ring, seq);                                              \
        else                                                                                    \
            hipLaunchKernelGGL((rollout_slots<L, B, false>), dim3(grid), dim3(B), 0, s, slots,   \
                               t, bad, ring, seq);                                              \
        return hipGetLastError();                                                               \
    }
    PLAN_LAUNCH(64)
    PLAN_LAUNCH(256)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace

// One-lane dispatch for launches of at most one wave per SIMD, defined in
// rollout_onelane_1wave.hip.
hipError_t launch_rollout_1wave(const RolloutArgs &a, int block, bool chunk, hipStream_t s);
hipError_t launch_sampled_1wave(const RolloutArgs &a, int block, hipStream_t s);
hipError_t launch_argmin_1wave(const RolloutArgs &a, int block, bool sampled, hipStream_t s);

// Two- and four-lane dispatch, defined in rollout_multilane.hip.
hipError_t launch_rollout_multi(const RolloutArgs &a, int lanes, int block, bool chunk,
                                hipStream_t s);
hipError_t launch_sampled_multi(const RolloutArgs &a, int lanes, int block, hipStream_t s);
hipError_t launch_ckpt_multi(const RolloutArgs &a, int lanes, int block, hipStream_t s);
hipError_t launch_argmin_multi(const RolloutArgs &a, int lanes, int block, bool sampled,
                               hipStream_t s);
hipError_t launch_slots_multi(const RolloutArgs *slots, const TickTable &t, int *bad,
                              SelectOut *ring, uint32_t seq, bool s1, int lanes, int block,
                              hipStream_t s);

}  // namespace plan
