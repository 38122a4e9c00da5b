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
constexpr int SM_CHUNK = 2048;                     // softmin: candidates per block
constexpr int SM_ROWS = 8;                         // softmin: plan entries per block

// --------------------------------------------------------------- terrain ----
// Node slopes by central differences (one-sided on the border), merged with
// the costmap into float4 texels (h, f_x, f_y, cost).
__global__ __launch_bounds__(256) void pack_terrain(const float *__restrict__ hgt,
                                                    const float *__restrict__ cm, int W, int H,
                                                    float inv_res, float4 *__restrict__ tex,
                                                    int *__restrict__ bad) {
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= W || j >= H) return;
    if (!pack_texel(hgt, cm, W, H, inv_res, i, j, tex)) atomicOr(bad, 1);
}

// ---------------------------------------------------------------- argmin ----
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Coherent read of a partial written by another block of the same launch.
__device__ __forceinline__ float load_partial(const float *p) {
    return __uint_as_float(__atomic_load_n((const unsigned int *)p, __ATOMIC_RELAXED));
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

// Softmin partial sums. Block (c, g) handles candidates [c*SM_CHUNK, ...) and
// plan rows [g*SM_ROWS, ...); row 2N is the weight sum. The last block to
// finish adds the chunk partials in chunk order and divides.
__global__ __launch_bounds__(SEL_BLOCK) void select_softmin(
    const float *__restrict__ cost, int K, const float *__restrict__ controls, int N,
    float drate_max, float inv_lambda, float *__restrict__ plan,
    float *__restrict__ wpart, unsigned int *__restrict__ ticket,
    const SelectOut *__restrict__ best) {
    __shared__ float w_sh[SM_CHUNK];
    __shared__ float red[SEL_BLOCK / 64][SM_ROWS + 1];
    __shared__ int last_sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int chunk = blockIdx.x, grp = blockIdx.y;
    const int nchunks = gridDim.x;
    const int rows = 2 * N + 1;
    const int k0 = chunk * SM_CHUNK;
    const int kn = min(SM_CHUNK, K - k0);
    const SelectOut bo = *best;
    const float jmin = bo.best_cost;
    const bool any = bo.best_k >= 0;
    for (int q = tid; q < SM_CHUNK; q += SEL_BLOCK) {
        float w = 0.0f;
        if (any && q < kn) {
            const float J = cost[k0 + q];
            if (isfinite(J)) w = __expf(-(J - jmin) * inv_lambda);
        }
        w_sh[q] = w;
    }
    __syncthreads();
    const int r0 = grp * SM_ROWS;
    for (int rr = 0; rr < SM_ROWS; ++rr) {
        const int r = r0 + rr;
        float acc = 0.0f;
        if (r < rows) {
            if (r == 2 * N) {
                for (int q = tid; q < kn; q += SEL_BLOCK) acc += w_sh[q];
            } else {
                const float *row = controls + (size_t)r * K + k0;
                for (int q = tid; q < kn; q += SEL_BLOCK)
                    acc += w_sh[q] * clamp_ctrl(row[q], r, drate_max);
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) red[wv][rr] = acc;
    }
    __syncthreads();
    if (tid < SM_ROWS) {
        const int r = r0 + tid;
        if (r < rows) {
            float s = 0.0f;
            for (int q = 0; q < SEL_BLOCK / 64; ++q) s += red[q][tid];
            wpart[(size_t)r * nchunks + chunk] = s;
        }
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        const unsigned int t = atomicAdd(ticket, 1u);
        last_sh = (t == gridDim.x * gridDim.y - 1);
    }
    __syncthreads();
    if (!last_sh) return;
    __threadfence();
    // last block: fixed-order sum over chunks, then divide by the weight sum
    float den = 0.0f;
    for (int c = 0; c < nchunks; ++c)
        den += load_partial(&wpart[(size_t)(2 * N) * nchunks + c]);
    for (int r = tid; r < 2 * N; r += SEL_BLOCK) {
        float num = 0.0f;
        for (int c = 0; c < nchunks; ++c)
            num += load_partial(&wpart[(size_t)r * nchunks + c]);
        plan[r] = any ? num / den : 0.0f;
    }
    if (tid == 0) *ticket = 0u;
}

}  // namespace

int select_blocks(int K) { return (K + SEL_CHUNK - 1) / SEL_CHUNK; }
int softmin_chunks(int K) { return (K + SM_CHUNK - 1) / SM_CHUNK; }
int softmin_row_groups(int N) { return (2 * N + 1 + SM_ROWS - 1) / SM_ROWS; }

hipError_t launch_pack_terrain(const float *h, const float *c, int W, int H, float inv_res,
                               float4 *tex, int *bad, hipStream_t s) {
    dim3 grid((W + 15) / 16, (H + 15) / 16);
    hipLaunchKernelGGL(pack_terrain, grid, dim3(256), 0, s, h, c, W, H, inv_res, tex, bad);
    return hipGetLastError();
}

hipError_t launch_select(int mode, float lambda, const float *controls, const float *cost,
                         int K, int N, float drate_max, float *plan_out,
                         unsigned long long *part_keys, unsigned int *counters, float *wpart,
                         SelectOut *out, SelectOut *out_host, uint32_t seq, hipStream_t s) {
    const int nb = select_blocks(K);
    hipLaunchKernelGGL(select_argmin<false>, dim3(nb), dim3(SEL_BLOCK), 0, s, cost, K, controls,
                       N, drate_max, mode == 0 ? 1 : 0, plan_out, part_keys, counters + 0, out,
                       out_host, seq, SampleArgs{});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || mode == 0) return e;
    dim3 grid(softmin_chunks(K), softmin_row_groups(N));
    hipLaunchKernelGGL(select_softmin, grid, dim3(SEL_BLOCK), 0, s, cost, K, controls, N,
                       drate_max, 1.0f / lambda, plan_out, wpart, counters + 1,
                       (const SelectOut *)out);
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
