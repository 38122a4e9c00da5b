// Terrain packing and candidate selection kernels (arXiv 2603.20525, section
// "Real-Time Implementation": costmap interpolated at run time, parallel
// argmin on the GPU, and the MPPI-style weighted average it is compared to).
//
// Selection is deterministic: the argmin reduces 64-bit keys
// (order-preserving cost bits << 32 | k), which makes the result independent
// of reduction order and breaks ties to the lowest k; the weighted average
// sums per fixed chunk and then over chunks in index order. Multi-block
// reductions finish in the last block to arrive (an atomic ticket), which
// resets the ticket for the next call, so no memset is needed between calls.
#include "plan_internal.h"
#include "select_common.h"

namespace plan {
namespace {

constexpr int SEL_BLOCK = 256;
constexpr int SEL_ITEMS = 16;                      // candidates per thread
constexpr int SEL_CHUNK = SEL_BLOCK * SEL_ITEMS;   // candidates per block
constexpr int SM_ROWS = 4;                         // softmin: plan entries per block
constexpr int SM_UNROLL = 8;                       // softmin: candidates in flight per thread
constexpr int SM_BLOCK = 1024;                     // softmin: threads per block

// --------------------------------------------------------------- terrain ----
// Node slopes by central differences (one-sided on the border), merged with
// the costmap, as the bilinear coefficients of each cell: one 16 x 16 tile
// of cells per workgroup (pack_tile).
__global__ __launch_bounds__(256) void pack_terrain(const float *__restrict__ hgt,
                                                    const float *__restrict__ cm, int W, int H,
                                                    float inv_res, float4 *__restrict__ cells,
                                                    int *__restrict__ bad) {
    __shared__ PackLds lds;
    if (!pack_tile(hgt, cm, W, H, inv_res, blockIdx.x * PACK_TILE, blockIdx.y * PACK_TILE,
                   cells, lds))
        atomicOr(bad, 1);
}

// ---------------------------------------------------------------- argmin ----
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One block per SEL_CHUNK candidates; each folds its minimum key into the
// slot part[0] (atomics only, see fold_key_and_take_ticket); the last block
// to arrive publishes (k*, J*) and, for argmin, writes the plan: from
// controls, or (SAMPLED) by regenerating candidate k*'s sequence.
template <bool SAMPLED>
__global__ __launch_bounds__(SEL_BLOCK) void select_argmin(
    const float *__restrict__ cost, int K, const float *__restrict__ controls, int N,
    float drate_max, int gather, float *__restrict__ plan,
    unsigned long long *__restrict__ part, unsigned int *__restrict__ ticket,
    SelectOut *__restrict__ out, SelectOut *out_host, uint32_t seq, const SampleArgs smp) {
    __shared__ unsigned long long red[SEL_BLOCK / 64];
    __shared__ int last_sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int base = blockIdx.x * SEL_CHUNK;
    unsigned long long key = ~0ull;
#pragma unroll
    for (int it = 0; it < SEL_ITEMS; ++it) {
        const int k = base + it * SEL_BLOCK + tid;
        if (k < K) {
            const unsigned long long kk = cost_key(cost[k], k);
            key = kk < key ? kk : key;
        }
    }
    key = wave_min(key);
    if (lane == 0) red[wv] = key;
    __syncthreads();
    if (tid == 0) {
        unsigned long long b = red[0];
        for (int q = 1; q < SEL_BLOCK / 64; ++q) b = red[q] < b ? red[q] : b;
        last_sh = fold_key_and_take_ticket(part, ticket, b, gridDim.x);
    }
    __syncthreads();
    if (!last_sh) return;
    if (tid == 0) {
        const unsigned long long m = take_key_and_reset(part, ticket);
        red[0] = m;
        // pinned host copy: no readback copy needed
        publish_result(out, out_host, m, seq, 0);
    }
    __syncthreads();
    if (gather) {
        const unsigned long long m = red[0];
        const int kb = (m == ~0ull) ? -1 : (int)(unsigned int)(m & 0xffffffffu);
        write_plan<SAMPLED>(kb, N, K, controls, smp, drate_max, plan, tid, SEL_BLOCK);
    }
}

// MPPI-style softmin in one launch with no traffic between workgroups.
// Workgroup g owns plan entries [g*SM_ROWS, (g+1)*SM_ROWS) of the 2N. Every
// workgroup takes the minimum key over all K itself (the costs are a few KB,
// served from L2), weighs each finite candidate w_k = exp(-(J_k - J_min) /
// lambda), and forms its entries' weighted sums of the clamped controls and
// the weight sum, each thread over a fixed stride of candidates and then in
// a fixed reduction tree, so the result does not depend on scheduling.
// Workgroup 0 publishes (k*, J*).
__global__ __launch_bounds__(SM_BLOCK) void select_softmin(
    const float *__restrict__ cost, int K, const float *__restrict__ controls, int N,
    float drate_max, float inv_lambda, float *__restrict__ plan, SelectOut *__restrict__ out,
    SelectOut *out_host, uint32_t seq) {
    __shared__ unsigned long long kred[SM_BLOCK / 64];
    __shared__ float fred[SM_BLOCK / 64][SM_ROWS + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    unsigned long long key = ~0ull;
    for (int k = tid; k < K; k += SM_BLOCK) {
        const unsigned long long kk = cost_key(cost[k], k);
        key = kk < key ? kk : key;
    }
    key = wave_min(key);
    if (lane == 0) kred[wv] = key;
    __syncthreads();
    unsigned long long m = kred[0];
#pragma unroll
    for (int q = 1; q < SM_BLOCK / 64; ++q) m = kred[q] < m ? kred[q] : m;
    if (blockIdx.x == 0 && tid == 0) publish_result(out, out_host, m, seq, 0);
    const bool any = m != ~0ull;
    const float jmin = any ? key_cost(m) : 0.0f;
    const int rows = 2 * N;
    const int r0 = blockIdx.x * SM_ROWS;
    float acc[SM_ROWS + 1];
#pragma unroll
    for (int j = 0; j <= SM_ROWS; ++j) acc[j] = 0.0f;
    if (any) {
        // SM_UNROLL candidates per thread per pass, all loads issued before
        // any is used; candidates still accumulate in the order k = tid,
        // tid + SM_BLOCK, ... for every thread
        for (int kb = tid; kb < K; kb += SM_BLOCK * SM_UNROLL) {
            float w[SM_UNROLL];
            float u[SM_ROWS][SM_UNROLL];
#pragma unroll
            for (int q = 0; q < SM_UNROLL; ++q) {
                const int k = kb + q * SM_BLOCK;
                const float J = k < K ? cost[k] : __builtin_inff();
#pragma unroll
                for (int j = 0; j < SM_ROWS; ++j) {
                    const int r = r0 + j;
                    u[j][q] = (k < K && r < rows) ? controls[(size_t)r * K + k] : 0.0f;
                }
                w[q] = isfinite(J) ? __expf(-(J - jmin) * inv_lambda) : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < SM_UNROLL; ++q) {
                acc[SM_ROWS] += w[q];
#pragma unroll
                for (int j = 0; j < SM_ROWS; ++j)
                    acc[j] += w[q] * clamp_ctrl(u[j][q], r0 + j, drate_max);
            }
        }
    }
#pragma unroll
    for (int j = 0; j <= SM_ROWS; ++j) {
        const float v = wave_sum(acc[j]);
        if (lane == 0) fred[wv][j] = v;
    }
    __syncthreads();
    if (tid < SM_ROWS && r0 + tid < rows) {
        float num = fred[0][tid], den = fred[0][SM_ROWS];
#pragma unroll
        for (int q = 1; q < SM_BLOCK / 64; ++q) {
            num += fred[q][tid];
            den += fred[q][SM_ROWS];
        }
        plan[r0 + tid] = any ? num / den : 0.0f;
    }
}

}  // namespace

int select_blocks(int K) { return (K + SEL_CHUNK - 1) / SEL_CHUNK; }

hipError_t launch_pack_terrain(const float *h, const float *c, int W, int H, float inv_res,
                               float4 *cells, int *bad, hipStream_t s) {
    dim3 grid((W + PACK_TILE - 1) / PACK_TILE, (H + PACK_TILE - 1) / PACK_TILE);
    hipLaunchKernelGGL(pack_terrain, grid, dim3(256), 0, s, h, c, W, H, inv_res, cells, bad);
    return hipGetLastError();
}

hipError_t launch_select(int mode, float lambda, const float *controls, const float *cost,
                         int K, int N, float drate_max, float *plan_out,
                         unsigned long long *part_keys, unsigned int *counters,
                         SelectOut *out, SelectOut *out_host, uint32_t seq, hipStream_t s) {
    if (mode == 0) {
        hipLaunchKernelGGL(select_argmin<false>, dim3(select_blocks(K)), dim3(SEL_BLOCK), 0, s,
                           cost, K, controls, N, drate_max, 1, plan_out, part_keys,
                           counters + 0, out, out_host, seq, SampleArgs{});
    } else {
        const unsigned groups = (unsigned)((2 * N + SM_ROWS - 1) / SM_ROWS);
        hipLaunchKernelGGL(select_softmin, dim3(groups), dim3(SM_BLOCK), 0, s, cost, K,
                           controls, N, drate_max, 1.0f / lambda, plan_out, out, out_host, seq);
    }
    return hipGetLastError();
}

hipError_t launch_select_sampled(const SampleArgs &sa, const float *cost, int K, int N,
                                 float drate_max, float *plan_out,
                                 unsigned long long *part_keys, unsigned int *counters,
                                 SelectOut *out, SelectOut *out_host, uint32_t seq,
                                 hipStream_t s) {
    const int nb = select_blocks(K);
    hipLaunchKernelGGL(select_argmin<true>, dim3(nb), dim3(SEL_BLOCK), 0, s, cost, K, nullptr, N,
                       drate_max, 1, plan_out, part_keys, counters + 0, out, out_host, seq, sa);
    return hipGetLastError();
}

}  // namespace plan
