// On-device candidate sampling (arXiv 2603.20525, section "Real-Time
// Implementation": the candidate control sequences are drawn on the GPU with
// a counter-based generator; the published configuration draws the steering
// rate uniformly and holds the longitudinal acceleration).
//
// Generator: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011). Candidate k, control interval n
// take the 64-bit word n mod 4 of the block at counter (k, n div 4, 0, 0)
// under the key (seed, stream). From that word w, a = bits 40..63 and
// b = bits 16..39 (24 bits each) give
//   uniform:  u_c = nominal_c + scale_c (2 x_c - 1), x_0 = a 2^-24, x_1 = b 2^-24
//   Gaussian: r = sqrt(-2 ln p), p = (a + 1) 2^-24, q = b 2^-24 (Box and
//             Muller, 1958): u_0 = nominal_0 + scale_0 r cos(2 pi q),
//             u_1 = nominal_1 + scale_1 r sin(2 pi q).
// With keep_nominal, candidate 0 is the nominal sequence itself. A candidate
// depends only on (seed, stream, k, n), so a sequence can be regenerated
// anywhere (the selection regenerates the winner instead of storing all K).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plan {

struct SampleArgs {
    int kind;            // PLAN_SAMPLE_UNIFORM or PLAN_SAMPLE_GAUSSIAN
    int keep_nominal;
    uint64_t key0, key1; // seed, stream
    float scale0, scale1;
    const float *nominal;  // [N][2] or nullptr (zeros)
};

struct PhiloxBlock {
    uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ PhiloxBlock philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                     uint64_t c3, uint64_t k0, uint64_t k1) {
    constexpr uint64_t MUL0 = 0xD2E7470EE14C6C93ull, MUL1 = 0xCA5A826395121157ull;
    constexpr uint64_t WEYL0 = 0x9E3779B97F4A7C15ull, WEYL1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(MUL0, c0), lo0 = MUL0 * c0;
        const uint64_t hi1 = __umul64hi(MUL1, c2), lo1 = MUL1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += WEYL0;
        k1 += WEYL1;
    }
    return PhiloxBlock{c0, c1, c2, c3};
}

__device__ __forceinline__ PhiloxBlock sample_block(const SampleArgs &sa, int k, int blk) {
    return philox4x64_10((uint64_t)(uint32_t)k, (uint64_t)(uint32_t)blk, 0, 0, sa.key0, sa.key1);
}

__device__ __forceinline__ uint64_t block_word(const PhiloxBlock &b, int j) {
    return j == 0 ? b.w0 : (j == 1 ? b.w1 : (j == 2 ? b.w2 : b.w3));
}

// Raw (unclamped) controls of candidate k at interval n from its word w.
__device__ __forceinline__ void draw_controls(const SampleArgs &sa, uint64_t w, int k, int n,
                                              float &u0, float &u1) {
    const float nom0 = sa.nominal ? sa.nominal[2 * n] : 0.0f;
    const float nom1 = sa.nominal ? sa.nominal[2 * n + 1] : 0.0f;
    if (sa.keep_nominal && k == 0) {
        u0 = nom0;
        u1 = nom1;
        return;
    }
    const float a = (float)(uint32_t)(w >> 40);
    const float b = (float)(uint32_t)((w >> 16) & 0xFFFFFFu);
    constexpr float TWO_M24 = 5.9604644775390625e-08f;  // 2^-24
    if (sa.kind == 0) {
        // 2 x - 1 is exact in FP32 for a 24-bit x
        const float t0 = 2.0f * (a * TWO_M24) - 1.0f;
        const float t1 = 2.0f * (b * TWO_M24) - 1.0f;
        u0 = nom0 + sa.scale0 * t0;
        u1 = nom1 + sa.scale1 * t1;
    } else {
        const float p = (a + 1.0f) * TWO_M24;
        const float q = b * TWO_M24;
        const float r = sqrtf(-2.0f * logf(p));
        float s, c;
        sincospif(2.0f * q, &s, &c);
        u0 = nom0 + sa.scale0 * (r * c);
        u1 = nom1 + sa.scale1 * (r * s);
    }
}

}  // namespace plan
