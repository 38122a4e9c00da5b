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
//   * Terrain: float4 texels (h, f_x, f_y, cost) on the heightmap grid;
//     software bilinear interpolation in FP32 with clamp-to-edge.
#include <string.h>

#include "plan_internal.h"
#include "rollout_step.h"
#include "select_common.h"

namespace plan {
namespace {

// One candidate k over control intervals [a.n0, a.n1), simulated by the
// LANES lanes of its group (this lane is number sub). CHUNK: start from and
// write back a.state / a.cost; otherwise start from a.s0 with zero cost and
// write a.cost / a.final_state. SAMPLED: draw the controls from a.smp (one
// generator block per four intervals, kept in registers) instead of reading
// a.controls. Lanes with store == false run a duplicate candidate only to
// keep their lane group complete.
template <int LANES, bool CHUNK, bool SAMPLED = false, bool RK4 = false, bool CKPT = false>
__device__ __forceinline__ float simulate(const RolloutArgs &a, int k, int sub, bool store) {
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
    bool done = false;

    const float *up = a.controls + k;
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

    for (int n = a.n0; n < a.n1 && !done; ++n) {
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
            u0 = up[(2 * (size_t)n) * K];
            u1 = up[(2 * (size_t)n + 1) * K];
        }
        const float dd = clampf_nan(u0, -a.drate_max, a.drate_max);
        const float ax = a.accel_max * clampf_nan(u1, -1.0f, 1.0f);

        for (int s = 0; s < a.S; ++s) {
            // goal test at the Euler node, before the step
            {
                const float gdx = st[0] - a.goal_x, gdy = st[1] - a.goal_y;
                if (fmaf(gdx, gdx, gdy * gdy) <= a.goal_r2) {
                    done = true;
                    break;
                }
            }
            if constexpr (RK4)
                rk4_step<LANES>(a, arms, st, J, dd, ax);
            else
                euler_step<LANES>(a, arms, st, J, dd, ax);
        }
        if constexpr (CKPT) {
            if ((n + 1) % a.ckpt_every == 0 && n + 1 < a.N) {
                ckpt_done = (n + 1) / a.ckpt_every;
                write_ckpt(ckpt_done);
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
// so the winner is the same as the separate selection kernel's); the last
// workgroup to arrive publishes (k*, J*), writes the plan and resets the key
// and the ticket for the next launch.
template <int BLOCK, bool SAMPLED>
__device__ __forceinline__ void argmin_epilogue(const RolloutArgs &a, unsigned long long key) {
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
        last_sh = fold_key_and_take_ticket(a.sel_key, a.sel_ticket, b, gridDim.x);
    }
    __syncthreads();
    if (!last_sh) return;
    if (tid == 0) {
        const unsigned long long m = take_key_and_reset(a.sel_key, a.sel_ticket);
        red[0] = m;
        SelectOut o;
        o.best_k = (m == ~0ull) ? -1 : (int)(unsigned int)(m & 0xffffffffu);
        o.best_cost = (m == ~0ull) ? __builtin_inff() : key_cost(m);
        o.pad[0] = o.pad[1] = 0;
        *a.sel_out = o;
        if (a.sel_out_host) *a.sel_out_host = o;
    }
    __syncthreads();
    const unsigned long long m = red[0];
    const int kb = (m == ~0ull) ? -1 : (int)(unsigned int)(m & 0xffffffffu);
    write_plan<SAMPLED>(kb, a.N, a.K, a.controls, a.smp, a.drate_max, a.plan, tid, BLOCK);
}

template <int LANES, int BLOCK, bool CHUNK, bool SAMPLED = false, bool FUSED = false,
          bool RK4 = false, bool CKPT = false>
__global__ __launch_bounds__(BLOCK) void rollout_srb(const RolloutArgs a) {
    const int gtid = blockIdx.x * BLOCK + threadIdx.x;
    const int sub = gtid & (LANES - 1);
    int k = gtid / LANES;
    const bool store = k < a.K;
    // Lanes past K simulate the last candidate again so that every lane group
    // is complete for the DPP sums; they store nothing (and reach the fused
    // epilogue's barriers like every other lane).
    if (!store) k = a.K - 1;
    const float J = simulate<LANES, CHUNK, SAMPLED, RK4, CKPT>(a, k, sub, store);
    if constexpr (FUSED)
        argmin_epilogue<BLOCK, SAMPLED>(a, (store && sub == 0) ? cost_key(J, k) : ~0ull);
}

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

// Several independent plans in one launch (the serving loop's tick). Entry e
// of the table owns blocks [e.block_start, next block_start) and advances
// slot e.slot through intervals [e.n0, e.n1); every block belongs to exactly
// one slot, so the per-slot arguments are wave-uniform.
template <int LANES, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rollout_slots(const RolloutArgs *__restrict__ slots,
                                                       const TickTable t) {
    int lo = 0, hi = t.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.e[mid].block_start <= (int)blockIdx.x)
            lo = mid;
        else
            hi = mid - 1;
    }
    const TickEntry te = t.e[lo];
    RolloutArgs a = slots[te.slot];
    a.n0 = te.n0;
    a.n1 = te.n1;
    a.finalize = te.finalize;
    const int gtid = ((int)blockIdx.x - te.block_start) * BLOCK + threadIdx.x;
    const int sub = gtid & (LANES - 1);
    int k = gtid / LANES;
    const bool store = k < a.K;
    if (!store) k = a.K - 1;
    simulate<LANES, true>(a, k, sub, store);
}

__global__ __launch_bounds__(256) void init_state(const RolloutArgs a) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= a.K) return;
#pragma unroll
    for (int q = 0; q < 13; ++q) a.state[(size_t)q * a.K + k] = a.s0[q];
    a.cost[k] = 0.0f;
}

}  // namespace

hipError_t launch_rollout(const RolloutArgs &a, int lanes, int block, bool chunk,
                          hipStream_t s) {
    const long long threads = (long long)a.K * lanes;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
#define PLAN_LAUNCH(L, B, C)                                                                   \
    if (lanes == L && block == B && chunk == C) {                                              \
        if (a.method == 1)                                                                     \
            hipLaunchKernelGGL((rollout_srb<L, B, C, false, false, true>), dim3(grid), dim3(B), \
                               0, s, a);                                                       \
        else                                                                                   \
            hipLaunchKernelGGL((rollout_srb<L, B, C>), dim3(grid), dim3(B), 0, s, a);          \
        return hipGetLastError();                                                              \
    }
    PLAN_LAUNCH(1, 64, false)
    PLAN_LAUNCH(2, 64, false)
    PLAN_LAUNCH(4, 64, false)
    PLAN_LAUNCH(1, 256, false)
    PLAN_LAUNCH(2, 256, false)
    PLAN_LAUNCH(4, 256, false)
    PLAN_LAUNCH(1, 64, true)
    PLAN_LAUNCH(2, 64, true)
    PLAN_LAUNCH(4, 64, true)
    PLAN_LAUNCH(1, 256, true)
    PLAN_LAUNCH(2, 256, true)
    PLAN_LAUNCH(4, 256, true)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_rollout_sampled(const RolloutArgs &a, int lanes, int block, hipStream_t s) {
    const long long threads = (long long)a.K * lanes;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
#define PLAN_LAUNCH(L, B)                                                                \
    if (lanes == L && block == B) {                                                      \
        hipLaunchKernelGGL((rollout_srb<L, B, false, true>), dim3(grid), dim3(B), 0, s, a); \
        return hipGetLastError();                                                        \
    }
    PLAN_LAUNCH(1, 64)
    PLAN_LAUNCH(2, 64)
    PLAN_LAUNCH(4, 64)
    PLAN_LAUNCH(1, 256)
    PLAN_LAUNCH(2, 256)
    PLAN_LAUNCH(4, 256)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_rollout_ckpt(const RolloutArgs &a, int lanes, int block, hipStream_t s) {
    const long long threads = (long long)a.K * lanes;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
#define PLAN_LAUNCH(L, B)                                                                      \
    if (lanes == L && block == B) {                                                            \
        hipLaunchKernelGGL((rollout_srb<L, B, false, false, false, false, true>), dim3(grid),  \
                           dim3(B), 0, s, a);                                                  \
        return hipGetLastError();                                                              \
    }
    PLAN_LAUNCH(1, 64)
    PLAN_LAUNCH(2, 64)
    PLAN_LAUNCH(4, 64)
    PLAN_LAUNCH(1, 256)
    PLAN_LAUNCH(2, 256)
    PLAN_LAUNCH(4, 256)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_rollout_argmin(const RolloutArgs &a, int lanes, int block, bool sampled,
                                 hipStream_t s) {
    const long long threads = (long long)a.K * lanes;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
#define PLAN_LAUNCH(L, B, SMP)                                                              \
    if (lanes == L && block == B && sampled == SMP) {                                       \
        hipLaunchKernelGGL((rollout_srb<L, B, false, SMP, true>), dim3(grid), dim3(B), 0, s, a); \
        return hipGetLastError();                                                           \
    }
    PLAN_LAUNCH(1, 64, false)
    PLAN_LAUNCH(2, 64, false)
    PLAN_LAUNCH(4, 64, false)
    PLAN_LAUNCH(1, 256, false)
    PLAN_LAUNCH(2, 256, false)
    PLAN_LAUNCH(4, 256, false)
    PLAN_LAUNCH(1, 64, true)
    PLAN_LAUNCH(2, 64, true)
    PLAN_LAUNCH(4, 64, true)
    PLAN_LAUNCH(1, 256, true)
    PLAN_LAUNCH(2, 256, true)
    PLAN_LAUNCH(4, 256, true)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_sample_controls(const SampleArgs &sa, int K, int N, float *controls,
                                  hipStream_t s) {
    const dim3 grid((unsigned)((K + 255) / 256), (unsigned)((N + 3) / 4));
    hipLaunchKernelGGL(sample_controls, grid, dim3(256), 0, s, sa, K, N, controls);
    return hipGetLastError();
}

hipError_t launch_rollout_slots(const RolloutArgs *slots, const TickTable &t, int lanes,
                                int block, hipStream_t s) {
    if (t.count < 1) return hipSuccess;
    const unsigned grid = (unsigned)t.total_blocks;
#define PLAN_LAUNCH(L, B)                                                              \
    if (lanes == L && block == B) {                                                    \
        hipLaunchKernelGGL((rollout_slots<L, B>), dim3(grid), dim3(B), 0, s, slots, t); \
        return hipGetLastError();                                                      \
    }
    PLAN_LAUNCH(1, 64)
    PLAN_LAUNCH(2, 64)
    PLAN_LAUNCH(4, 64)
    PLAN_LAUNCH(1, 256)
    PLAN_LAUNCH(2, 256)
    PLAN_LAUNCH(4, 256)
#undef PLAN_LAUNCH
    return hipErrorInvalidValue;
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
