// Counter-based normal noise for the SGLD update.
//
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds, each multiplying words 0 and 2 by
// fixed 32-bit multipliers, keeping the low halves as the new words 1 and 3
// and xoring the high halves with the other two words and the round key into
// the new words 0 and 2; the two key words advance by fixed Weyl increments
// between rounds.  Normals by the Box-Muller transform on pairs of words:
// u = ((w >> 9) + 1/2) 2^-23 (exact in FP32, never 0 or 1),
// z0 = sqrt(-2 ln u_a) cos(2 pi u_b), z1 = sqrt(-2 ln u_a) sin(2 pi u_b).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgs {

__host__ __device__ inline uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * x.x, p1 = (uint64_t)0xCD9E8D57u * x.z;
        x = make_uint4((uint32_t)(p1 >> 32) ^ x.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ x.w ^ k1, (uint32_t)p0);
    }
    return x;
}

// ((w >> 8) + 1/2) 2^-24: a uniform in (0, 1), exact in FP32.
__host__ __device__ inline float uniform24(uint32_t w) {
    return ((float)(w >> 8) + 0.5f) * 5.9604644775390625e-08f;
}

// floor(w n / 2^32): an integer uniform over [0, n) from a word, exact.
__host__ __device__ inline uint32_t choice32(uint32_t w, uint32_t n) {
    return (uint32_t)(((uint64_t)w * n) >> 32);
}

__device__ inline void box_muller_pair(uint32_t wa, uint32_t wb, float& z0, float& z1) {
    const float ua = ((float)(wa >> 9) + 0.5f) * 1.1920928955078125e-07f;
    const float ub = ((float)(wb >> 9) + 0.5f) * 1.1920928955078125e-07f;
    const float r = sqrtf(-2.0f * logf(ua));
    float s, c;
    sincospif(2.0f * ub, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// The four normals of counter (index lo, index hi, tag, step) under `seed`.
__device__ inline void normals4(uint64_t index, uint32_t tag, uint32_t step, uint64_t seed, float z[4]) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)index, (uint32_t)(index >> 32), tag, step), (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    box_muller_pair(w.x, w.y, z[0], z[1]);
    box_muller_pair(w.z, w.w, z[2], z[3]);
}

// Noise streams (tags): per Gaussian of scene s, tag 0x10000 s (normals: mean
// x, y, z, opacity logit); codebook row k of scene s, row-layout column c,
// counter index 16 k + c / 4, tag 0x10000 s + 1, normal c % 4.
__device__ inline uint32_t gaussian_tag(int scene) { return 0x10000u * (uint32_t)scene; }
__device__ inline uint32_t codebook_tag(int scene) { return 0x10000u * (uint32_t)scene + 1u; }

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ inline uint16_t f32_to_bf16_rne(float f) {
    const uint32_t b = __float_as_uint(f);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40u);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

}  // namespace cgs
