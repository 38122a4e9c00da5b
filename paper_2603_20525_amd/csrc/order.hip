// Candidate order for gather locality.
//
// A one-lane rollout wave runs 64 candidates side by side, and every step
// each lane gathers the terrain cells under its own four wheels. Candidates drawn
// independently end up tens of metres apart, so a single gather instruction
// touches up to 64 different cache lines and the texture path (address unit
// and L1), not the vector ALUs, sets the pace at large K. Running candidates
// with similar trajectories in the same wave restores locality. The order
// only decides which lane simulates which candidate: every candidate's
// arithmetic, its outputs and the selection are unchanged.
//
// The order comes from a cheap kinematic proxy of each candidate (single-track
// kinematics with the control limits of the model and a friction-limited
// curvature), whose lateral offsets from the start at a quarter, half,
// three quarters and the end of the horizon are interleaved bit by bit into
// a 32-bit Morton key and sorted with a stable LSD radix sort (four 8-bit
// digits; per digit: tile histograms, one scan, a stable scatter).
#include "plan_internal.h"

namespace plan {
namespace {

constexpr int ORDER_TILE = 1024;       // elements per scatter workgroup (256 threads x 4)
constexpr int ORDER_BLOCK = 256;
static_assert(ORDER_BLOCK == 256, "the scatter scans the 256 digit totals with one thread each");
constexpr int ORDER_PROXY_SUB = 4;     // proxy substeps per control interval (at most)
constexpr int ORDER_PROXY_STEPS = 64;  // about this many proxy substeps over the horizon
// proxy workgroups: large, so that few atomics per value fold the range
// (same-address atomics from every workgroup serialise)
constexpr int ORDER_PROXY_BLOCK = 1024;

// IEEE float <-> unsigned with the same order (for atomic min / max).
__device__ __forceinline__ unsigned float_to_ordered(float f) {
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ordered_to_float(unsigned u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void order_reset(OrderArgs o) {
    if (threadIdx.x < 8) o.range[threadIdx.x] = threadIdx.x < 4 ? 0xffffffffu : 0u;
}

// Proxy trajectory of candidate k: lateral offsets after intervals
// (m+1) N / 4 - 1, m = 0..3; their range goes to o.range by atomic min / max.
template <bool SAMPLED>
__global__ __launch_bounds__(ORDER_PROXY_BLOCK) void order_proxy(OrderArgs o) {
    __shared__ float red[8][ORDER_PROXY_BLOCK / 64];
    const int k = blockIdx.x * ORDER_PROXY_BLOCK + threadIdx.x;
    float lat[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const bool active = k < o.K;
    if (active) {
        const size_t K = (size_t)o.K;
        float d = o.delta0, v = o.vx0, psi = 0.0f, y = 0.0f;
        // long horizons take fewer substeps per interval: the proxy only ranks
        const int sub = max(1, min(ORDER_PROXY_SUB, ORDER_PROXY_STEPS / o.N));
        const float h = o.dt / (float)sub;
        PhiloxBlock blk{};
        int m = 0;
        for (int n = 0; n < o.N; ++n) {
            float u0, u1;
            if constexpr (SAMPLED) {
                if ((n & 3) == 0) blk = sample_block(o.smp, k, n >> 2);
                draw_controls(o.smp, block_word(blk, n & 3), k, n, u0, u1);
            } else {
                u0 = o.controls[(2 * (size_t)n) * K + k];
                u1 = o.controls[(2 * (size_t)n + 1) * K + k];
            }
            u0 = fminf(fmaxf(u0, -o.drate_max), o.drate_max);
            u1 = fminf(fmaxf(u1, -1.0f), 1.0f);
            d = fminf(fmaxf(d + u0 * o.dt, -o.delta_max), o.delta_max);
            v = fmaxf(v + o.accel_max * u1 * o.dt, o.vx_min);
            const float klim = o.mu_g / fmaxf(v * v, 1e-6f);
            const float kap = fminf(fmaxf(tanf(d) * o.inv_wheelbase, -klim), klim);
            for (int s = 0; s < sub; ++s) {
                psi += v * kap * h;
                y += v * __sinf(psi) * h;
            }
            while (m < 4 && n == ((m + 1) * o.N) / 4 - 1) lat[m++] = y;
        }
        while (m < 4) lat[m++] = y;  // N < 4
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!isfinite(lat[q])) lat[q] = 0.0f;
            o.lat[(size_t)q * o.lat_stride + k] = lat[q];
        }
    }
    // block min / max of the four offsets, then one atomic per value
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float lo = active ? lat[q] : __builtin_inff();
        float hi = active ? lat[q] : -__builtin_inff();
        for (int off = 32; off > 0; off >>= 1) {
            lo = fminf(lo, __shfl_xor(lo, off));
            hi = fmaxf(hi, __shfl_xor(hi, off));
        }
        if (lane == 0) {
            red[q][wv] = lo;
            red[4 + q][wv] = hi;
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int q = threadIdx.x;
        float r = red[q][0];
        for (int w = 1; w < ORDER_PROXY_BLOCK / 64; ++w)
            r = q < 4 ? fminf(r, red[q][w]) : fmaxf(r, red[q][w]);
        if (isfinite(r)) {
            if (q < 4)
                atomicMin(&o.range[q], float_to_ordered(r));
            else
                atomicMax(&o.range[q], float_to_ordered(r));
        }
    }
}

// Morton key of the quantised offsets (8 bits each, the earliest offset in
// the most significant position of each group).
__global__ __launch_bounds__(ORDER_BLOCK) void order_keys(OrderArgs o) {
    const int k = blockIdx.x * ORDER_BLOCK + threadIdx.x;
    if (k >= o.K) return;
    unsigned q[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const float lo = ordered_to_float(o.range[m]);
        const float hi = ordered_to_float(o.range[4 + m]);
        const float span = hi - lo;
        const float x = o.lat[(size_t)m * o.lat_stride + k];
        float t = span > 0.0f ? (x - lo) * (256.0f / span) : 0.0f;
        t = fminf(fmaxf(t, 0.0f), 255.0f);
        q[m] = (unsigned)t;
    }
    unsigned key = 0u;
#pragma unroll
    for (int b = 7; b >= 0; --b)
#pragma unroll
        for (int m = 0; m < 4; ++m) key = (key << 1) | ((q[m] >> b) & 1u);
    o.keys[0][k] = key;
    o.vals[0][k] = k;
}

// Histogram of digit p over one tile of the current order: hist[d nt + tile]
// (every entry written, so the table needs no clearing between passes).
__global__ __launch_bounds__(ORDER_BLOCK) void order_hist(OrderArgs o, int p) {
    __shared__ unsigned cnt[256];
    cnt[threadIdx.x] = 0u;
    __syncthreads();
    const unsigned *kin = o.keys[p & 1];
    const int base = blockIdx.x * ORDER_TILE;
    const int shift = 8 * p;
#pragma unroll
    for (int r = 0; r < ORDER_TILE / ORDER_BLOCK; ++r) {
        const int pos = base + r * ORDER_BLOCK + threadIdx.x;
        if (pos < o.K) atomicAdd(&cnt[(kin[pos] >> shift) & 255u], 1u);
    }
    __syncthreads();
    const int nt = (o.K + ORDER_TILE - 1) / ORDER_TILE;
    o.hist[(size_t)threadIdx.x * nt + blockIdx.x] = cnt[threadIdx.x];
}

// Per-digit exclusive scan of hist[digit][tile] over the tiles (in place)
// and the digit's total: one wave per digit, 64 tiles per step.
__global__ __launch_bounds__(ORDER_BLOCK) void order_scan(OrderArgs o) {
    const int lane = threadIdx.x & 63;
    const int d = blockIdx.x * (ORDER_BLOCK / 64) + (threadIdx.x >> 6);
    const int nt = (o.K + ORDER_TILE - 1) / ORDER_TILE;
    unsigned *h = o.hist + (size_t)d * nt;
    unsigned carry = 0u;
    for (int t0 = 0; t0 < nt; t0 += 64) {
        const int t = t0 + lane;
        const unsigned c = t < nt ? h[t] : 0u;
        unsigned x = c;  // inclusive scan over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (t < nt) h[t] = carry + x - c;
        carry += __shfl(x, 63);
    }
    if (lane == 0) o.dtotal[d] = carry;
}

// Stable scatter of one tile by digit p. The digits' output bases come from
// an exclusive scan of the 256 digit totals, the tile's start within each
// digit from the per-digit scan. Each wave ranks its 256 elements in four
// rounds of 64: the lanes holding the same digit are found with eight
// ballots, and a per-wave, per-digit count in LDS carries the rank across
// rounds. The last pass writes only the candidate order and resets the
// offset range for the next call.
__global__ __launch_bounds__(ORDER_BLOCK) void order_scatter(OrderArgs o, int p) {
    __shared__ unsigned cnt[ORDER_BLOCK / 64][256];
    __shared__ unsigned dbase[256], wtot[ORDER_BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int src = p & 1;
    const unsigned *kin = o.keys[src];
    const int *vin = o.vals[src];
    unsigned *kout = o.keys[src ^ 1];
    int *vout = o.vals[src ^ 1];
    const unsigned *off = o.hist;
    const int nt = (o.K + ORDER_TILE - 1) / ORDER_TILE;
    const int tile = blockIdx.x;
    const int shift = 8 * p;
    for (int i = threadIdx.x; i < (ORDER_BLOCK / 64) * 256; i += ORDER_BLOCK)
        (&cnt[0][0])[i] = 0u;
    {
        // exclusive scan of the digit totals (ORDER_BLOCK = 256 threads, one per digit)
        const unsigned c = o.dtotal[threadIdx.x];
        unsigned x = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wtot[wv] = x;
        __syncthreads();
        unsigned before = 0u;
        for (int w = 0; w < wv; ++w) before += wtot[w];
        dbase[threadIdx.x] = before + x - c;
    }
    __syncthreads();

    constexpr int R = ORDER_TILE / ORDER_BLOCK;  // rounds per wave
    unsigned key[R];
    int val[R];
    unsigned rank[R];
    const int wbase = tile * ORDER_TILE + wv * (64 * R);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int pos = wbase + r * 64 + lane;
        const bool valid = pos < o.K;
        key[r] = valid ? kin[pos] : 0u;
        val[r] = valid ? vin[pos] : 0;
        const unsigned d = (key[r] >> shift) & 255u;
        unsigned long long peer = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long bb = __ballot((d >> b) & 1u);
            peer &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const unsigned below = __builtin_amdgcn_mbcnt_hi(
            (unsigned)(peer >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)peer, 0u));
        const unsigned base = cnt[wv][d];
        rank[r] = base + below;
        // the highest lane of each digit group advances the digit's count
        if (valid && (peer >> lane) == 1ull) cnt[wv][d] = base + (unsigned)__popcll(peer);
    }
    __syncthreads();
    {
        // per-digit start of each wave's elements in the output
        const int d = threadIdx.x;
        unsigned run = dbase[d] + off[(size_t)d * nt + tile];
#pragma unroll
        for (int w = 0; w < ORDER_BLOCK / 64; ++w) {
            const unsigned c = cnt[w][d];
            cnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int pos = wbase + r * 64 + lane;
        if (pos >= o.K) continue;
        const unsigned d = (key[r] >> shift) & 255u;
        const unsigned dest = cnt[wv][d] + rank[r];
        if (dest >= (unsigned)o.K) continue;  // unreachable for consistent histograms
        vout[dest] = val[r];
        if (p < 3) kout[dest] = key[r];
    }
    if (p == 3 && tile == 0 && threadIdx.x < 8)
        o.range[threadIdx.x] = threadIdx.x < 4 ? 0xffffffffu : 0u;
}

__global__ __launch_bounds__(ORDER_BLOCK) void permute_controls(const float *__restrict__ u,
                                                              const int *__restrict__ order,
                                                              int K, int rows,
                                                              float *__restrict__ out) {
    const long long i = (long long)blockIdx.x * ORDER_BLOCK + threadIdx.x;
    if (i >= (long long)rows * K) return;
    const int row = (int)(i / K), slot = (int)(i % K);
    const int k = min(max(order[slot], 0), K - 1);
    out[i] = u[(size_t)row * K + k];
}

}  // namespace

hipError_t launch_permute_controls(const float *controls, const int *order, int K, int N,
                                   float *out, hipStream_t s) {
    const long long n = 2ll * N * K;
    hipLaunchKernelGGL(permute_controls, dim3((unsigned)((n + ORDER_BLOCK - 1) / ORDER_BLOCK)),
                       dim3(ORDER_BLOCK), 0, s, controls, order, K, 2 * N, out);
    return hipGetLastError();
}

int order_tiles(int max_K) { return (max_K + ORDER_TILE - 1) / ORDER_TILE; }

hipError_t launch_order_reset(const OrderArgs &o, hipStream_t s) {
    hipLaunchKernelGGL(order_reset, dim3(1), dim3(64), 0, s, o);
    return hipGetLastError();
}

hipError_t launch_locality_order(const OrderArgs &o, hipStream_t s) {
    if (o.K < 1 || o.K > o.lat_stride || order_tiles(o.K) > o.nt_max) return hipErrorInvalidValue;
    const unsigned gp = (unsigned)((o.K + ORDER_PROXY_BLOCK - 1) / ORDER_PROXY_BLOCK);
    if (o.controls)
        hipLaunchKernelGGL((order_proxy<false>), dim3(gp), dim3(ORDER_PROXY_BLOCK), 0, s, o);
    else
        hipLaunchKernelGGL((order_proxy<true>), dim3(gp), dim3(ORDER_PROXY_BLOCK), 0, s, o);
    const unsigned gk = (unsigned)((o.K + ORDER_BLOCK - 1) / ORDER_BLOCK);
    hipLaunchKernelGGL(order_keys, dim3(gk), dim3(ORDER_BLOCK), 0, s, o);
    const unsigned nt = (unsigned)order_tiles(o.K);
    for (int p = 0; p < 4; ++p) {
        hipLaunchKernelGGL(order_hist, dim3(nt), dim3(ORDER_BLOCK), 0, s, o, p);
        hipLaunchKernelGGL(order_scan, dim3(256 / (ORDER_BLOCK / 64)), dim3(ORDER_BLOCK), 0, s, o);
        hipLaunchKernelGGL(order_scatter, dim3(nt), dim3(ORDER_BLOCK), 0, s, o, p);
    }
    return hipGetLastError();
}

}  // namespace plan
