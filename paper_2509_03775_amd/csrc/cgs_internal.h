// Internal declarations of libcgs: the device-side batch descriptor, the
// workspace plan and wave64 helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cgs.h"

namespace cgs {

constexpr int kTile = 16;               // tile edge in pixels
constexpr int kWave = 64;               // CDNA wavefront width
constexpr int kSortItems = 16;          // keys per lane in the radix/scan kernels
constexpr int kSortBlock = 256;         // threads per radix/scan workgroup
constexpr int kSortTile = kSortItems * kSortBlock;   // keys per workgroup (4096)
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kReduceChunk = 64;        // sorted positions owned by one reduction wavefront
constexpr int kMaxRowWidth = 8 + 48;    // ls3 q4 logit1 + degree-3 SH
constexpr uint32_t kCulledKey = 0x7f800000u;   // +inf bits: sorts after every depth
constexpr float kClampFov = 1.3f;       // Jacobian clamp, in half-fields of view
// One blend record per (view, Gaussian): 48 B, i.e. three float4 at rec[3r]:
//   [0] (u, v, -A/2 log2e, -B log2e)   [1] (-C/2 log2e, opacity, red, green)
//   [2] (blue, tile rect lo, tile rect hi, first gradient slot within the
//   record's 64-record chunk).  No padding to 64 B: the preprocess writes a
//   quarter less, and the blends' gathers (half of them now straddling two
//   64-byte segments) come from L2 and are not what bounds the blends.
constexpr int kRecF4 = 3;

// ---------------------------------------------------------------- descriptors
struct ViewDesc {
    int32_t W, H, tiles_x, tiles_y;
    int32_t scene, scene_vi;   // the scene, and this view's place among the scene's views
    int64_t tile_off, pix_off, rec_off;
    int64_t rec_wave_off;   // wavefronts before this view when records are split view-aligned
    float fx, fy, cx, cy;
    // Jacobian clamp limits of the tangents, kClampFov * (W/2) / fx and the
    // same in y, in FP32 as the skeleton takes them (set by the host)
    float limx, limy;
    float Rt[12];
    float campos[3];
    float bg[3];
};

struct SceneDesc {
    int64_t n, g_off;
    int64_t wave_off;       // wavefronts before this scene when Gaussians are split scene-aligned
    // The nonzero flags of the records' gradients (two words per record
    // wavefront) are stored Gaussian-major within a scene: wavefront q of the
    // scene's vi-th view at flag_wave_off + q*vcount + vi, so the flags of one
    // Gaussian's views share a line.
    int64_t flag_wave_off;
    int64_t sr_rows, sh_rows, sr_row_off, sh_row_off;
    const float* means;
    const int32_t* idx_sr;
    const int32_t* idx_sh;
    const void* sr;
    const void* sh;
    const float* opacity;
    int32_t sr_stride, sr_col0, sh_stride, sh_col0;
    int32_t opacity_mode, vfirst, vcount, fused;
    float* g_means;
    float* g_sr;
    float* g_sh;
    float* g_opacity;
    int32_t g_sr_stride, g_sr_col0, g_sh_stride, g_sh_col0;
    // SGLD update targets (FP32 masters; see cgs_scene_params)
    float* u_means;
    float* u_opacity;
    float* u_sr;
    float* u_sh;
    int32_t u_sr_stride, u_sr_col0, u_sh_stride, u_sh_col0;
};

struct BatchDesc {
    int32_t n_views, n_scenes, sh_degree, dtype;
    int32_t row_width;      // 8 + 3 (d+1)^2: per-Gaussian gradient row
    int32_t tile_order;
    int32_t vec_rows;       // every codebook row is 16-byte aligned: vector loads allowed
    int32_t pack_rect;      // every view is below 256 tiles per side: rectangles fit one word
    const uint32_t* tile_perm;   // tile order 2: tiles by descending list length
    int64_t n_rec, n_gauss, n_tiles, n_pix, capacity;
    int64_t sr_rows_total, sh_rows_total;
    int64_t n_gauss_waves, n_rec_waves;   // scene-aligned / view-aligned wavefront counts
    // SGLD update fused into the backward (sgld != 0): step sizes of means,
    // opacity logit, SR columns, SH columns; Philox key and step
    int32_t sgld, step;
    float eps[4];
    uint64_t seed;
    int32_t view_list[CGS_MAX_VIEWS];   // views grouped by scene
    ViewDesc views[CGS_MAX_VIEWS];
    SceneDesc scenes[CGS_MAX_SCENES];
};

// Image geometry of a batch of views for the loss kernels (by value).
struct LossViews {
    int32_t n;
    int32_t H[CGS_MAX_VIEWS], W[CGS_MAX_VIEWS], tiles_x[CGS_MAX_VIEWS];
    int64_t pix_off[CGS_MAX_VIEWS];
    int64_t tile_off[CGS_MAX_VIEWS + 1];
};

// Arguments and workspace of the Metropolis-Hastings codebook moves.
struct MhArgs {
    float* rows;
    int64_t ld, D, K_max, n;
    int64_t* d_rows;
    int32_t* idx;
    uint16_t* mirror;
    int64_t mirror_ld;
    float lambda, inv_s2, inv_m2;   // lambda, 1/eps_split^2, 1/eps_merge^2
    float eps_split;
    int64_t B;
    uint64_t seed;
    uint32_t step;
};
struct MhWs {
    uint32_t *mark, *acc, *s0, *s1, *valid, *rank, *partner, *flag, *scan, *hole_of, *fin;
    float* u;
    unsigned long long *tot, *bsum;
};

constexpr int kQueues = 8;          // tile queues of a persistent blend (one per XCD)
constexpr int kQueueStride = 16;    // u64 words between queues (128 bytes)

// Device counters kept in the workspace.
struct DevCounters {
    unsigned long long n_inst;     // instances needed
    unsigned long long n_inst_ok;  // instances emitted (0 on overflow)
    unsigned long long done_fwd, done_bwd;   // retired wavefronts of the persistent blends
    unsigned long long pad[4];
    // tile queues of the persistent blends, one per XCD (workgroups are
    // dispatched to the 8 XCDs round-robin), each on its own 128-byte line:
    // queue x hands out positions x, x + 8, x + 16, ... of the tile order.
    // Zeroed by the forward's capacity check and reset by the last wavefront
    // of each persistent launch.
    unsigned long long q_fwd[kQueues * kQueueStride];
    unsigned long long q_bwd[kQueues * kQueueStride];
};

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------ wave helpers
__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// Orders LDS traffic of one wavefront (all lanes run in lockstep; the fences
// keep the compiler from moving LDS accesses across the point).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t popc_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// Sum over the 64 lanes (every lane must be active); result valid in all lanes.
// DPP row shifts build 16-lane sums, row broadcasts combine rows; the total
// lands in lane 63 and is read back as a wave-uniform value.
__device__ inline float wave_sum(float v) {
    int x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum over the 64 lanes into lane 63 (every lane must be active): row sums
// by DPP shifts, then lane 15 of each row into the next row, then lane 31
// into rows 2-3, giving ((r3 + r2) + (r1 + r0)) in lane 63 (other lanes hold
// partial sums; the broadcasts use all row masks so each step is one fused
// DPP add).
__device__ inline float wave_sum_to_63(float v) {
    int x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xf, 0xf, true));   // row_bcast:15
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xf, 0xf, true));   // row_bcast:31
    __asm__ volatile("" : "+v"(v));
    return v;
}

// Sum of each aligned group of 8 lanes, in the group's last lane (lanes
// 8m + 7); the other lanes hold partial sums.  Every lane must be active.
__device__ inline float group8_sum_to_last(float v) {
    int x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));  // row_shr:4
    __asm__ volatile("" : "+v"(v));
    return v;
}

// Bitwise OR over the 64 lanes (every lane must be active); valid in all lanes.
__device__ inline uint32_t wave_or_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v |= (uint32_t)__shfl_xor((int)v, d, 64);
    return v;
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t o = (uint32_t)__shfl_xor((int)v, d, 64);
        v = v > o ? v : o;
    }
    return v;
}

// Inclusive prefix sum over the wave (u32).
__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane) {
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

template <int DT>
__device__ inline float load_cb(const void* p, int64_t i) {
    if constexpr (DT == CGS_BF16) return bf16_to_f32(static_cast<const uint16_t*>(p)[i]);
    else return static_cast<const float*>(p)[i];
}

// Wavefront index within the launch, wave-uniform (scalar) by construction.
__device__ inline int64_t wave_id(int waves_per_block) {
    return (int64_t)blockIdx.x * waves_per_block + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Per-Gaussian kernels give each wavefront 64 Gaussians of one scene, so
// the scene (and its views) are wave-uniform and their descriptors are read
// with scalar loads.  Last scene whose first wavefront is <= w.
__device__ inline int find_scene_by_wave(const BatchDesc* d, int64_t w) {
    int lo = 0, hi = d->n_scenes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d->scenes[mid].wave_off <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Same for per-record kernels: 64 records of one view per wavefront.
__device__ inline int find_view_by_wave(const BatchDesc* d, int64_t w) {
    int lo = 0, hi = d->n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d->views[mid].rec_wave_off <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int find_scene(const BatchDesc* d, int64_t g) {
    int lo = 0, hi = d->n_scenes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d->scenes[mid].g_off <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int find_view_by_tile(const BatchDesc* d, int64_t t) {
    int lo = 0, hi = d->n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d->views[mid].tile_off <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int find_view_by_rec(const BatchDesc* d, int64_t r) {
    int lo = 0, hi = d->n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d->views[mid].rec_off <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------- launchers
// (defined in the .hip files; all enqueue on `st` and never synchronise)
hipError_t upload_bytes(void* dst, const void* src, size_t n, hipStream_t st);
// Two byte ranges (whole words each) uploaded by one launch when they fit
// 2 KB together, else by upload_bytes each.
hipError_t upload_two(void* dst_a, const void* src_a, size_t na, void* dst_b, const void* src_b, size_t nb,
                      hipStream_t st);
hipError_t fill_u32(void* dst, uint32_t value, size_t count, hipStream_t st);

// Exclusive scan of n u32 values read through `perm` (NULL = identity):
// out[j] = sum_{i<j} in[perm[i]]; *total = sum of all (u64).
// zeroed: the scan's tile states (scan_states) were zeroed beforehand.
hipError_t scan_u32(const uint32_t* in, const uint32_t* perm, int64_t n, uint32_t* out,
                    unsigned long long* total, unsigned long long* bsum, hipStream_t st, bool zeroed = false);

// Up to four spans of u32 words a kernel zeroes on its way, so that the sorts
// and scans after it need no fill launches of their own (unused spans: n 0).
struct ZeroSpans {
    uint32_t* p[4];
    uint32_t n[4];
};
// The words a radix sort over n_max items in `ws` (digit counts, tickets,
// depth range), or a one-pass scan of n items in `bsum` (tile states), zeroes
// before it starts; a caller that zeroes them beforehand passes zeroed = true.
uint32_t* sort_counters(void* ws, int64_t n_max, uint32_t* count);
uint32_t* scan_states(unsigned long long* bsum, int64_t n, uint32_t* count);

// Stable LSD radix sort of (key, value) u32 pairs on bits [0, nbits), at
// most 32 bits.  The first pass reads kin/vin (vin NULL: value = position),
// later passes ping-pong between kbuf/vbuf[0] and [1] (kin may alias
// kbuf[1]).  n_dev (optional) holds the live item count, clamped to n_max.
// ws: radix_ws_bytes(n_max) bytes of scratch.  Returns the index (0/1) of
// the buffer pair that holds the result.
// last (optional) makes the final pass write each item's tile rectangle
// (rect_out, packed u16 x0,y0 | x1,y1, half open) and tile count (cnt_out),
// either gathered through the value (rect_in[value]) or, when pay_in is set,
// from a packed payload word (x0 | y0 << 8 | x1 << 16 | y1 << 24, tiles below
// 256 per side) that every pass carries with the item (pay_in read by the
// first pass, pay_buf[2] in between).  With drop_keys the final pass writes
// no keys.
struct SortGather {
    const uint2* rect_in;
    uint2* rect_out;
    uint32_t* cnt_out;
    int drop_keys;
    const uint32_t* pay_in;
    uint32_t* pay_buf[2];
};
size_t radix_ws_bytes(int64_t n_max);
int radix_sort_pairs(const uint32_t* kin, const uint32_t* vin, uint32_t* kbuf[2], uint32_t* vbuf[2], int64_t n_max,
                     const unsigned long long* n_dev, int nbits, void* ws, hipStream_t st, hipError_t* err,
                     const SortGather* last = nullptr, bool zeroed = false);
// The records' depth sort with the packed-rectangle payload (g.pay_in,
// g.pay_buf): 9-bit digits over the keys relative to the live depth range
// (from krange: n_part pairs (max ~key, max key) over live keys),
// only the passes the range needs; results in kbuf/vbuf[1], g.rect_out and
// g.cnt_out.  Returns 1.
int radix_sort_depth(const uint32_t* kin, const uint32_t* krange, int64_t n_part, uint32_t* kbuf[2], uint32_t* vbuf[2],
                     int64_t n, void* ws, hipStream_t st, hipError_t* err, const SortGather& g,
                     bool zeroed = false);
// Look-back waits of the radix passes that hit their bound on the current
// device since the library was loaded (synchronous read; 0 expected).
uint32_t sort_stalls();

hipError_t tile_len_keys(const uint32_t* ranges, int64_t n_tiles, uint32_t* key, hipStream_t st);

// Workgroups of `kernel` (a __global__ function) at `block` threads that the
// current device holds at once: CUs x the occupancy its registers and LDS
// allow (the grid of a persistent launch); 0 if the query fails.  Cached per
// (device, kernel, block).
int64_t resident_blocks(const void* kernel, int block);

hipError_t tile_ranges(const uint32_t* sorted_tile, const unsigned long long* n_dev, int64_t n_max,
                       int64_t n_tiles, uint32_t* ranges, hipStream_t st);
// The same over 16-bit tile keys (batches of at most 65536 tiles), and the
// radix sort of 16-bit keys with 32-bit values (plain passes only).
hipError_t tile_ranges16(const uint16_t* sorted_tile, const unsigned long long* n_dev, int64_t n_max,
                         int64_t n_tiles, uint32_t* ranges, hipStream_t st);
int radix_sort_pairs16(const uint16_t* kin, const uint32_t* vin, uint16_t* kbuf[2], uint32_t* vbuf[2], int64_t n_max,
                       const unsigned long long* n_dev, int nbits, void* ws, hipStream_t st, hipError_t* err,
                       bool zeroed = false);

}  // namespace cgs
