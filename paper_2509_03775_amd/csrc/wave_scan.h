// Wave-level scan used by the wave-cooperative kernels (emission, slot sums).
#pragma once
#include "cgs_internal.h"

namespace cgs {

// Inclusive max over lanes 0..l of the wave (values >= 0, every lane active):
// prefixes within each 16-lane row by DPP row shifts, then the totals of the
// rows before it, read from lanes 15, 31 and 47.
__device__ inline uint32_t wave_incl_max_u32(uint32_t v, int lane) {
    uint32_t t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v = v > t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v = v > t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v = v > t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v = v > t ? v : t;
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    const uint32_t m01 = r0 > r1 ? r0 : r1, m012 = m01 > r2 ? m01 : r2;
    const int row = lane >> 4;
    const uint32_t pre = row == 0 ? 0u : (row == 1 ? r0 : (row == 2 ? m01 : m012));
    return v > pre ? v : pre;
}

// Inclusive sum over lanes 0..l of the wave (every lane active), the same
// way: row prefixes by DPP row shifts, then the totals of the earlier rows.
__device__ inline uint32_t wave_incl_sum_u32(uint32_t v, int lane) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    const int row = lane >> 4;
    const uint32_t pre = row == 0 ? 0u : (row == 1 ? r0 : (row == 2 ? r0 + r1 : r0 + r1 + r2));
    return v + pre;
}

}  // namespace cgs
