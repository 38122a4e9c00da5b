// Device helpers shared by the selection kernels and the rollout kernel's
// fused argmin epilogue (section "Real-Time Implementation": the sampled
// candidate of minimal cost is the plan).
//
// The argmin reduces 64-bit keys (order-preserving cost bits << 32 | k): the
// minimum of a set of keys does not depend on the order in which it is taken,
// so any reduction tree gives the same winner, and equal costs resolve to the
// lowest k. Non-finite costs map to the largest key and are never selected.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan_internal.h"
#include "sample.h"

namespace plan {

__device__ __forceinline__ unsigned long long cost_key(float J, int k) {
    if (!isfinite(J)) return ~0ull;
    unsigned int b = __float_as_uint(J);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // order-preserving
    return ((unsigned long long)b << 32) | (unsigned int)k;
}

__device__ __forceinline__ float key_cost(unsigned long long key) {
    unsigned int b = (unsigned int)(key >> 32);
    b = (b & 0x80000000u) ? (b & 0x7fffffffu) : ~b;
    return __uint_as_float(b);
}

__device__ __forceinline__ unsigned long long wave_min(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

// The selection result: a device copy, and (optional) the pinned host copy
// written as two 16-byte stores, (k*, seq, J*, seq) and (status, seq, 0, 0).
// Nothing orders the two stores as the host sees them, so every 8-byte word
// the host reads carries seq.
__device__ __forceinline__ void publish_result(SelectOut *out, SelectOut *out_host,
                                               unsigned long long m, uint32_t seq,
                                               int32_t status) {
    SelectOut o;
    o.best_k = (m == ~0ull) ? -1 : (int)(unsigned int)(m & 0xffffffffu);
    o.best_cost = (m == ~0ull) ? __builtin_inff() : key_cost(m);
    o.seq_k = o.seq_cost = o.seq_status = seq;
    o.status = status;
    o.pad[0] = o.pad[1] = 0u;
    *out = o;
    if (out_host) {
        uint4 *h = reinterpret_cast<uint4 *>(out_host);
        h[0] = make_uint4((unsigned int)o.best_k, seq, __float_as_uint(o.best_cost), seq);
        h[1] = make_uint4((unsigned int)status, seq, 0u, 0u);
    }
}

// Admissible-set clamp of plan row `row` ([N][2] flattened: even rows are
// steering rates, odd rows throttle).
__device__ __forceinline__ float clamp_ctrl(float u, int row, float drate_max) {
    const float lim = (row & 1) ? 1.0f : drate_max;
    return u < -lim ? -lim : (u > lim ? lim : u);
}

// Cross-workgroup argmin without memory fences. Each workgroup folds its
// minimum key into *slot with an atomic minimum and then takes a ticket; the
// ticket increment is made data-dependent on the minimum's returned value, so
// it is issued only after the minimum has been performed. The workgroup that
// draws the last ticket reads the slot with an atomic (every other
// workgroup's minimum was performed before its ticket) and resets slot and
// ticket for the next launch. Only atomics cross workgroups, so no cache
// writeback or invalidation is needed (a fence would write back and
// invalidate the whole L2 of each XCD). Called by one thread per workgroup;
// returns whether this workgroup is the last.
__device__ __forceinline__ bool fold_key_and_take_ticket(unsigned long long *slot,
                                                         unsigned int *ticket,
                                                         unsigned long long key,
                                                         unsigned int nblocks) {
    // keys are never 0 (that would be a NaN cost), so the increment is 1
    const unsigned long long old = atomicMin(slot, key);
    const unsigned int t = atomicAdd(ticket, old == 0ull ? 2u : 1u);
    return t == nblocks - 1;
}

// The last workgroup's read of the folded key, with the reset for the next
// launch (slot all ones, ticket zero).
__device__ __forceinline__ unsigned long long take_key_and_reset(unsigned long long *slot,
                                                                 unsigned int *ticket) {
    const unsigned long long m = atomicExch(slot, ~0ull);
    atomicExch(ticket, 0u);
    return m;
}

// Plan output [N][2] for the selected candidate kb (zeros if kb < 0): its
// clamped controls, read from controls [N][2][K] or, SAMPLED, regenerated
// from the generator. Threads tid, tid + nthreads, ... share the work.
template <bool SAMPLED>
__device__ __forceinline__ void write_plan(int kb, int N, int K, const float *controls,
                                           const SampleArgs &smp, float drate_max, float *plan,
                                           int tid, int nthreads) {
    if constexpr (SAMPLED) {
        for (int n = tid; n < N; n += nthreads) {
            float u0 = 0.0f, u1 = 0.0f;
            if (kb >= 0) {
                const PhiloxBlock blk = sample_block(smp, kb, n >> 2);
                draw_controls(smp, block_word(blk, n & 3), kb, n, u0, u1);
                u0 = clamp_ctrl(u0, 0, drate_max);
                u1 = clamp_ctrl(u1, 1, drate_max);
            }
            plan[2 * n] = u0;
            plan[2 * n + 1] = u1;
        }
    } else {
        // the column gather is one scattered load per plan entry: each thread
        // issues four before it stores any, so their latencies overlap
        constexpr int B = 4;
        for (int e0 = tid; e0 < 2 * N; e0 += B * nthreads) {
            float v[B];
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int e = e0 + q * nthreads;
                v[q] = (kb >= 0 && e < 2 * N) ? controls[(size_t)e * K + kb] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int e = e0 + q * nthreads;
                if (e < 2 * N) plan[e] = (kb < 0) ? 0.0f : clamp_ctrl(v[q], e, drate_max);
            }
        }
    }
}

}  // namespace plan
