// Integer primitives of the binning stage: descriptor upload, fills,
// exclusive scan and a stable LSD radix sort of (u32 key, u32 value) pairs.
// All of it is bit-exact integer work.
//
// Radix sort layout: a workgroup of 256 threads owns 4096 consecutive items;
// wave w owns items [w*1024, w*1024+1024) and walks them 64 at a time, so the
// item order inside a workgroup is (wave, step, lane) and ranks computed in
// that order keep the sort stable.  Lanes holding equal digits find each
// other with one ballot per digit bit; the lowest of them updates the wave's
// running count in LDS.  Counts are laid out digit-major ([digit][block]) so a
// single exclusive scan yields every (digit, block) output offset.
#include "cgs_internal.h"

namespace cgs {

// ------------------------------------------------------------------ upload
struct UploadChunk {
    uint32_t words[256];
};

__global__ void k_upload(uint32_t* dst, UploadChunk c, int nwords) {
    int t = threadIdx.x;
    if (t < nwords) dst[t] = c.words[t];
}

hipError_t upload_bytes(void* dst, const void* src, size_t n, hipStream_t st) {
    const uint32_t* s = static_cast<const uint32_t*>(src);
    uint32_t* d = static_cast<uint32_t*>(dst);
    size_t words = (n + 3) / 4;
    for (size_t off = 0; off < words; off += 256) {
        UploadChunk c;
        int nw = (int)((words - off) < 256 ? (words - off) : 256);
        for (int i = 0; i < nw; ++i) {
            size_t b = (off + i) * 4;
            uint32_t w = 0;
            size_t take = n - b < 4 ? n - b : 4;
            __builtin_memcpy(&w, reinterpret_cast<const char*>(s) + b, take);
            c.words[i] = w;
        }
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, st, d + off, c, nw);
    }
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* dst, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = v;
}

hipError_t fill_u32(void* dst, uint32_t value, size_t count, hipStream_t st) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<uint32_t*>(dst), value, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------- scan
__device__ inline uint32_t scan_load(const uint32_t* in, const uint32_t* perm, int64_t i) {
    return perm ? in[perm[i]] : in[i];
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int i = 0; i < kSortBlock / 64; ++i) {
        uint32_t x = s_wave[i];
        if (i < w) before += x;
        all += x;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(kSortBlock) void k_scan_reduce(const uint32_t* in, const uint32_t* perm, int64_t n,
                                                            unsigned long long* bsum) {
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    unsigned long long acc = 0;
    for (int i = 0; i < kSortItems; ++i) {
        int64_t j = base + (int64_t)i * kSortBlock + threadIdx.x;
        if (j < n) acc += scan_load(in, perm, j);
    }
    __shared__ unsigned long long s[kSortBlock];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int d = kSortBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

// Exclusive scan of nb block sums in place by one workgroup; total -> *total.
__global__ __launch_bounds__(1024) void k_scan_blocks(unsigned long long* bsum, int64_t nb,
                                                      unsigned long long* total) {
    __shared__ unsigned long long s[1024];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t j = base + threadIdx.x;
        unsigned long long v = j < nb ? bsum[j] : 0ull;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            unsigned long long t = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0ull;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (j < nb) bsum[j] = carry + s[threadIdx.x] - v;
        unsigned long long blk = s[1023];
        __syncthreads();
        carry += blk;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kSortBlock) void k_scan_down(const uint32_t* in, const uint32_t* perm, int64_t n,
                                                          const unsigned long long* bsum, uint32_t* out) {
    __shared__ uint32_t s_wave[kSortBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    uint32_t carry = (uint32_t)bsum[blockIdx.x];
    uint32_t v[kSortItems];      // all loads issued before the first barrier
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t j = base + (int64_t)i * kSortBlock + threadIdx.x;
        v[i] = j < n ? scan_load(in, perm, j) : 0u;
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t j = base + (int64_t)i * kSortBlock + threadIdx.x;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v[i], s_wave, &tot);
        if (j < n) out[j] = carry + ex;
        carry += tot;
    }
}

hipError_t scan_u32(const uint32_t* in, const uint32_t* perm, int64_t n, uint32_t* out,
                    unsigned long long* total, unsigned long long* bsum, hipStream_t st) {
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb == 0) {
        if (total) hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bsum, (int64_t)0, total);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kSortBlock), 0, st, in, perm, n, bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kSortBlock), 0, st, in, perm, n, bsum, out);
    return hipGetLastError();
}

// ------------------------------------------------------------- radix sort
__device__ inline int64_t live_count(int64_t n_max, const unsigned long long* n_dev) {
    if (!n_dev) return n_max;
    unsigned long long v = *n_dev;
    return (int64_t)v < n_max ? (int64_t)v : n_max;
}

// Mask of active lanes whose digit (< 2^kRadixBits) equals this lane's:
// one ballot per digit bit (bits above a narrower pass's width are zero and
// match trivially).
__device__ inline uint64_t match_digit(uint32_t d) {
    uint64_t peers = __ballot(1);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint32_t bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint32_t* keys, int64_t n_max,
                                                           const unsigned long long* n_dev, int shift, int nbits,
                                                           uint32_t* counts, int64_t nblocks) {
    __shared__ uint32_t hist[kRadixBins];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = live_count(n_max, n_dev);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * (kSortTile / 4);
    const uint32_t mask = (1u << nbits) - 1u;
    if ((int64_t)blockIdx.x * kSortTile < n) {
        uint32_t k_[kSortItems];     // all loads issued before the first LDS update
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const int64_t j = base + i * 64 + lane;
            k_[i] = j < n ? keys[j] : 0u;
        }
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const int64_t j = base + i * 64 + lane;
            if (j < n) {
                const uint32_t d = (k_[i] >> shift) & mask;
                const uint64_t peers = match_digit(d);
                if (popc_below(peers) == 0) atomicAdd(&hist[d], (uint32_t)__popcll(peers));
            }
        }
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

// Scatter pass.  Ranks are computed per wave in item order as in the
// histogram pass; the workgroup then places its items in LDS in block-local
// digit order and writes them out linearly, so each digit's run of items goes
// to consecutive global addresses (coalesced) instead of 64 scattered writes
// per instruction.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const uint32_t* keys_in, const uint32_t* vals_in,
                                                              uint32_t* keys_out, uint32_t* vals_out,
                                                              int64_t n_max, const unsigned long long* n_dev,
                                                              int shift, int nbits, const uint32_t* offsets,
                                                              int64_t nblocks) {
    __shared__ uint32_t cnt[4][kRadixBins];
    __shared__ uint32_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t s_goff[kRadixBins];
    __shared__ uint32_t s_wave[kSortBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = 0; i < 4; ++i) cnt[i][threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = live_count(n_max, n_dev);
    const int64_t blk0 = (int64_t)blockIdx.x * kSortTile;
    if (blk0 >= n) return;     // whole workgroup: nothing here
    const int64_t base = blk0 + (int64_t)w * (kSortTile / 4);
    const uint32_t mask = (1u << nbits) - 1u;
    uint32_t k_[kSortItems], v_[kSortItems];
    uint32_t rank[kSortItems];
    // all loads issued before the first LDS update
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t j = base + i * 64 + lane;
        k_[i] = j < n ? keys_in[j] : 0u;
        v_[i] = j < n ? (vals_in ? vals_in[j] : (uint32_t)j) : 0u;
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        int64_t j = base + i * 64 + lane;
        rank[i] = 0xffffffffu;
        if (j < n) {
            const uint32_t key = k_[i];
            uint32_t d = (key >> shift) & mask;
            uint64_t peers = match_digit(d);
            uint32_t below = popc_below(peers);
            uint32_t run = cnt[w][d];
            rank[i] = run + below;
            wave_sync();
            if (below == 0) cnt[w][d] = run + (uint32_t)__popcll(peers);
        }
        wave_sync();
    }
    __syncthreads();
    // per digit: block-local start (prefix over digits), each wave's local
    // base, and the shift from local to global positions
    {
        const uint32_t d = threadIdx.x;
        uint32_t tot = 0, wb[4];
        for (int i = 0; i < 4; ++i) { wb[i] = tot; tot += cnt[i][d]; }
        uint32_t all;
        const uint32_t dstart = block_excl_scan(tot, s_wave, &all);
        for (int i = 0; i < 4; ++i) cnt[i][d] = dstart + wb[i];
        s_goff[d] = offsets[(int64_t)d * nblocks + blockIdx.x] - dstart;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (rank[i] != 0xffffffffu) {
            const uint32_t d = (k_[i] >> shift) & mask;
            const uint32_t lp = cnt[w][d] + rank[i];
            s_key[lp] = k_[i];
            s_val[lp] = v_[i];
        }
    }
    __syncthreads();
    const int m = (int)(n - blk0 < kSortTile ? n - blk0 : kSortTile);
    for (int i = threadIdx.x; i < m; i += kSortBlock) {
        const uint32_t key = s_key[i];
        const uint32_t pos = s_goff[(key >> shift) & mask] + (uint32_t)i;
        keys_out[pos] = key;
        vals_out[pos] = s_val[i];
    }
}

int radix_sort_pairs(const uint32_t* kin, const uint32_t* vin, uint32_t* kbuf[2], uint32_t* vbuf[2], int64_t n_max,
                     const unsigned long long* n_dev, int nbits, uint32_t* counts, unsigned long long* bsum,
                     hipStream_t st, hipError_t* err) {
    *err = hipSuccess;
    const int passes = (nbits + kRadixBits - 1) / kRadixBits;
    const int final_buf = passes > 0 ? (passes - 1) & 1 : 0;
    const int64_t nblocks = (n_max + kSortTile - 1) / kSortTile;
    if (nblocks == 0 || nbits <= 0) return final_buf;
    const uint32_t* ksrc = kin;
    const uint32_t* vsrc = vin;
    int out = 0;
    for (int shift = 0; shift < nbits; shift += kRadixBits) {
        const int pb = nbits - shift < kRadixBits ? nbits - shift : kRadixBits;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblocks), dim3(kSortBlock), 0, st, ksrc, n_max, n_dev, shift,
                           pb, counts, nblocks);
        hipError_t e = scan_u32(counts, nullptr, nblocks * kRadixBins, counts, nullptr, bsum, st);
        if (e != hipSuccess) { *err = e; return final_buf; }
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblocks), dim3(kSortBlock), 0, st, ksrc, vsrc, kbuf[out],
                           vbuf[out], n_max, n_dev, shift, pb, counts, nblocks);
        ksrc = kbuf[out];
        vsrc = vbuf[out];
        out ^= 1;
    }
    *err = hipGetLastError();
    return final_buf;
}

// ----------------------------------------------------------- tile ranges
// ranges[t] = [lower_bound(t), lower_bound(t+1)) over the sorted tile keys.
__global__ void k_tile_ranges(const uint32_t* sorted, const unsigned long long* n_dev, int64_t n_max,
                              int64_t n_tiles, uint32_t* ranges) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const int64_t n = live_count(n_max, n_dev);
    auto lower = [&](uint64_t key) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((uint64_t)sorted[mid] < key) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    ranges[2 * t] = (uint32_t)lower((uint64_t)t);
    ranges[2 * t + 1] = (uint32_t)lower((uint64_t)t + 1);
}

// Sort key of each tile for the heavy-first order: 0xffff - min(length, 0xffff).
__global__ void k_tile_len_keys(const uint32_t* ranges, int64_t n_tiles, uint32_t* key) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    key[t] = 0xffffu - (len < 0xffffu ? len : 0xffffu);
}

hipError_t tile_len_keys(const uint32_t* ranges, int64_t n_tiles, uint32_t* key, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_len_keys, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, st, ranges, n_tiles,
                       key);
    return hipGetLastError();
}

hipError_t tile_ranges(const uint32_t* sorted_tile, const unsigned long long* n_dev, int64_t n_max,
                       int64_t n_tiles, uint32_t* ranges, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, st,
                       sorted_tile, n_dev, n_max, n_tiles, ranges);
    return hipGetLastError();
}

}  // namespace cgs
