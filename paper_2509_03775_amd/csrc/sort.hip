// Integer primitives of the binning stage: descriptor upload, fills,
// exclusive scan and a stable LSD radix sort of (u32 key, u32 value) pairs.
// All of it is bit-exact integer work.
//
// Radix sort layout: a workgroup of 512 threads owns a tile of 8192
// consecutive items and ranks them in item order, so the sort is stable;
// per-tile digit states are published tile-major ([tile][digit], 64-bit
// words: a 2-bit state, how far back the sum reaches, the sum) for the
// look-back.
#include <mutex>

#include "cgs_internal.h"
#include "wave_scan.h"

namespace cgs {

// ------------------------------------------------------------------ upload
struct UploadChunk {
    uint32_t words[256];
};

__global__ void k_upload(uint32_t* dst, UploadChunk c, int nwords) {
    int t = threadIdx.x;
    if (t < nwords) dst[t] = c.words[t];
}

// Two destinations in one launch: words [0, na) to a, [na, nw) to b.
struct UploadPair {
    uint32_t words[512];
};

__global__ void k_upload2(uint32_t* a, uint32_t* b, UploadPair c, int na, int nw) {
    for (int t = threadIdx.x; t < nw; t += blockDim.x) {
        if (t < na) a[t] = c.words[t];
        else b[t - na] = c.words[t];
    }
}

// Whole words of src (n a multiple of 4) into c.words from position at.
static void pack_words(UploadPair& c, size_t at, const void* src, size_t n) {
    __builtin_memcpy(&c.words[at], src, n);
}

hipError_t upload_two(void* dst_a, const void* src_a, size_t na, void* dst_b, const void* src_b, size_t nb,
                      hipStream_t st) {
    const size_t wa = na / 4, wb = nb / 4;
    if (na % 4 != 0 || nb % 4 != 0 || wa + wb > 512) {
        hipError_t e = upload_bytes(dst_a, src_a, na, st);
        return e == hipSuccess ? upload_bytes(dst_b, src_b, nb, st) : e;
    }
    if (wa + wb == 0) return hipSuccess;
    UploadPair c;
    pack_words(c, 0, src_a, na);
    pack_words(c, wa, src_b, nb);
    hipLaunchKernelGGL(k_upload2, dim3(1), dim3(256), 0, st, static_cast<uint32_t*>(dst_a),
                       static_cast<uint32_t*>(dst_b), c, (int)wa, (int)(wa + wb));
    return hipGetLastError();
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

hipError_t scan_onepass(const uint32_t* in, int64_t n, uint32_t* out, unsigned long long* total,
                        unsigned long long* bsum, hipStream_t st, bool zeroed);

hipError_t scan_u32(const uint32_t* in, const uint32_t* perm, int64_t n, uint32_t* out,
                    unsigned long long* total, unsigned long long* bsum, hipStream_t st, bool zeroed) {
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb == 0) {
        if (total) hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bsum, (int64_t)0, total);
        return hipGetLastError();
    }
    if (!perm) return scan_onepass(in, n, out, total, bsum, st, zeroed);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kSortBlock), 0, st, in, perm, n, bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kSortBlock), 0, st, in, perm, n, bsum, out);
    return hipGetLastError();
}

// ------------------------------------------------------------- radix sort
// Single-pass form of the LSD radix sort (decoupled look-back, Merrill &
// Garland 2016; one sweep per digit, Adinets & Merrill 2022).  k_os_hist
// counts the digits of every pass from the input keys at once (a digit
// histogram does not depend on the order of the keys).  Each pass is then one
// kernel: a workgroup takes a ticket (its tile of kOsTile items, in the order
// workgroups start), ranks its items, publishes its per-digit counts and
// walks back over the states of tiles with earlier tickets.  A state holds a
// sum of counts and how far back it reaches: "tiles (k, t]" while tile t is
// still walking (it is rewritten at each step, so a tile behind it can jump
// over the stretch t has already summed), "tiles [0, t]" once t is done.  A
// ticket is taken only by a running workgroup and a workgroup publishes its
// state before it waits, so every wait ends; the wait is still bounded (a
// stall is counted and the pass finishes with its writes kept in bounds).
//
// The depth sort of the records uses 9-bit digits over keys relative to the
// batch's depth range: k_key_range finds the least and largest live depth key,
// a key becomes min(key, largest) - least (culled records, whose key is +inf,
// take the largest live key: they own no instances, so their place in the
// order is never read), and only the passes that cover the range's bits run
// (three for a range under 2^27); the last of them writes the final buffers.
constexpr int kOsThreads = 512;             // 8 waves
constexpr int kOsWaves = kOsThreads / 64;
constexpr int kOsItems = 16;                // keys per lane
constexpr int kOsTile = kOsItems * kOsThreads;   // 8192 keys per workgroup (the smallest tile: workspaces are sized by it)
// 16-bit keys take 20 per lane: a digit's run in a 10240-key tile is about
// 80 bytes of keys instead of 64, fewer partial-line writes per pass
template <typename KT>
constexpr int os_items() { return sizeof(KT) == 2 ? 20 : kOsItems; }
constexpr int kOsHistBlocks = 512;
constexpr int kDepthBits = 9;               // digit width of the depth sort
constexpr int kMaxBins = 1 << kDepthBits;
constexpr uint64_t kStAgg = 1ull << 62;     // bits 32..61: k + 1; low 32: count of tiles (k, t]
constexpr uint64_t kStInc = 2ull << 62;     // low 32: count of tiles [0, t]
constexpr uint32_t kSpinLimit = 1u << 21;

__device__ uint32_t g_sort_stalls;          // bounded waits that gave up since load

__device__ inline int64_t live_count(int64_t n_max, const unsigned long long* n_dev) {
    if (!n_dev) return n_max;
    unsigned long long v = *n_dev;
    return (int64_t)v < n_max ? (int64_t)v : n_max;
}

__device__ inline void status_put(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t status_get(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int RB>
__device__ inline uint32_t pass_mask(int nbits, int p) {
    const int w = nbits - p * RB < RB ? nbits - p * RB : RB;
    return (1u << w) - 1u;
}

// The depth range: range[0] = ~(least live key), range[1] = largest live key
// (both start at 0, both found by atomicMax).
struct DepthRange {
    uint32_t lo, hi;
    bool any;
};

__device__ inline DepthRange depth_range(const uint32_t* range) {
    DepthRange r;
    r.lo = ~range[0];
    r.hi = range[1];
    r.any = r.lo <= r.hi;
    return r;
}

__device__ inline uint32_t depth_rel(uint32_t key, const DepthRange& r) {
    if (!r.any) return 0u;
    return (key < r.hi ? key : r.hi) - r.lo;
}

// Passes the depth range needs (at least one).
__device__ inline int depth_passes(const DepthRange& r) {
    const uint32_t span = r.any ? r.hi - r.lo : 0u;
    const int bits = span == 0u ? 1 : 32 - __clz(span);
    return (bits + kDepthBits - 1) / kDepthBits;
}

// The depth range from per-wavefront partials (pairs: max of ~key, max of key
// over the wavefront's live keys, written by the preprocessing).
__global__ __launch_bounds__(256) void k_key_range(const uint2* part, int64_t n_part, uint32_t* range) {
    uint32_t nlo = 0u, hi = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_part; i += (int64_t)gridDim.x * 256) {
        const uint2 pr = part[i];
        nlo = pr.x > nlo ? pr.x : nlo;
        hi = pr.y > hi ? pr.y : hi;
    }
    nlo = wave_max_u32(nlo);
    hi = wave_max_u32(hi);
    __shared__ uint32_t s_lo[4], s_hi[4];
    if ((threadIdx.x & 63) == 0) { s_lo[threadIdx.x >> 6] = nlo; s_hi[threadIdx.x >> 6] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) { nlo = s_lo[w] > nlo ? s_lo[w] : nlo; hi = s_hi[w] > hi ? s_hi[w] : hi; }
        if (nlo) atomicMax(&range[0], nlo);
        if (hi) atomicMax(&range[1], hi);
    }
}

// Exclusive scan over the workgroup of one value per thread (kOsThreads).
__device__ inline uint32_t os_scan(uint32_t v, uint32_t* s_wave) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < kOsWaves; ++i)
        if (i < w) before += s_wave[i];
    __syncthreads();
    return before + inc - v;
}

// Single-pass exclusive scan (decoupled look-back, Merrill & Garland 2016):
// a 512-thread workgroup takes a ticket (its tile of 8192 consecutive items,
// in start order), sums its items, publishes its total, and wave 0 looks
// back over 64 earlier tiles' states at a time until one holds an inclusive
// prefix; each wave reads and writes its 1024 items 64 at a time (DPP wave
// scans with a running carry).  st[0] is the
// ticket counter and st[1 + t] tile t's state (2-bit flag, 62-bit sum), all
// zero on entry.  Offsets are u32 (they wrap only past 2^32 instances, which
// the capacity check rejects on the exact 64-bit total).
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanItems * kOsThreads;
constexpr uint64_t kStVal = (1ull << 62) - 1ull;

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, 64);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

__global__ __launch_bounds__(kOsThreads) void k_scan_1p(const uint32_t* in, int64_t n, uint32_t* out,
                                                        unsigned long long* total, unsigned long long* st) {
    __shared__ uint32_t s_wave[kOsWaves];
    __shared__ unsigned long long s_wsum[kOsWaves];
    __shared__ unsigned long long s_excl;
    __shared__ uint32_t s_ticket;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_ticket = (uint32_t)atomicAdd(&st[0], 1ull);
    __syncthreads();
    const int64_t b = s_ticket;
    // wave w owns items [1024 w, 1024 w + 1024) of the tile, read 64 at a time
    const int64_t wbase = b * kScanTile + (int64_t)w * (kScanItems * 64);
    uint32_t v[kScanItems], inc[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t j = wbase + i * 64 + lane;
        v[i] = j < n ? in[j] : 0u;
    }
    uint32_t carry = 0;
    unsigned long long wtot = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const uint32_t x = wave_incl_sum_u32(v[i], lane);
        inc[i] = carry + x;
        const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
        carry += t;
        wtot += t;
    }
    if (lane == 0) { s_wave[w] = carry; s_wsum[w] = wtot; }
    __syncthreads();
    uint32_t woff = 0;
#pragma unroll
    for (int i = 0; i < kOsWaves; ++i)
        if (i < w) woff += s_wave[i];
    if (w == 0) {
        unsigned long long tot = 0;
#pragma unroll
        for (int i = 0; i < kOsWaves; ++i) tot += s_wsum[i];
        uint64_t* const sts = reinterpret_cast<uint64_t*>(st + 1);   // tile states
        uint64_t* mine = sts + b;
        if (lane == 0) status_put(mine, (b == 0 ? kStInc : kStAgg) | tot);
        unsigned long long excl = 0;
        int64_t k = b - 1;
        uint32_t spins = 0;
        while (k >= 0) {
            const int64_t kk = k - lane;              // lane 0: the nearest earlier tile
            const uint64_t sk = kk >= 0 ? status_get(sts + kk) : kStInc;
            const uint64_t f = sk >> 62;
            const uint64_t incm = __ballot(f == 2), pending = __ballot(f == 0);
            const int first = incm ? (int)__builtin_ctzll(incm) : 64;
            const uint64_t need = first < 63 ? (2ull << first) - 1ull : ~0ull;
            if (pending & need) {
                if (++spins >= kSpinLimit) {
                    if (lane == 0) atomicAdd(&g_sort_stalls, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += wave_sum_u64(lane <= first ? (sk & kStVal) : 0ull);
            if (first < 64) break;
            k -= 64;
        }
        if (lane == 0) {
            if (b > 0) status_put(mine, kStInc | (excl + tot));
            s_excl = excl;
            if ((b + 1) * kScanTile >= n && total) *total = excl + tot;
        }
    }
    __syncthreads();
    const uint32_t base = (uint32_t)s_excl + woff;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t j = wbase + i * 64 + lane;
        if (j < n) out[j] = base + inc[i] - v[i];
    }
}

uint32_t* scan_states(unsigned long long* bsum, int64_t n, uint32_t* count) {
    *count = (uint32_t)(2 * ((n + kScanTile - 1) / kScanTile + 1));
    return reinterpret_cast<uint32_t*>(bsum);
}

hipError_t scan_onepass(const uint32_t* in, int64_t n, uint32_t* out, unsigned long long* total,
                        unsigned long long* bsum, hipStream_t st, bool zeroed) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipError_t e = zeroed ? hipSuccess : fill_u32(bsum, 0u, 2 * (size_t)(nb + 1), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_1p, dim3((unsigned)nb), dim3(kOsThreads), 0, st, in, n, out, total, bsum);
    return hipGetLastError();
}

struct SortWs {
    uint64_t* status[2];    // [tiles][bins] per pass, the two alternating
    uint32_t* ghist;        // [4][bins] digit counts of every pass
    uint32_t* tickets;      // [4] per pass
    uint32_t* range;        // [2] the depth sort's key range
};

// Laid out for the widest digit (the 8-bit sorts use the front of each row).
SortWs sort_ws(void* ws, int64_t n_max) {
    const int64_t nb = std::max<int64_t>(1, (n_max + kOsTile - 1) / kOsTile);
    char* p = static_cast<char*>(ws);
    SortWs s;
    const size_t st_bytes = align_up(8 * (size_t)kMaxBins * (size_t)nb);
    s.status[0] = reinterpret_cast<uint64_t*>(p);
    s.status[1] = reinterpret_cast<uint64_t*>(p + st_bytes);
    s.ghist = reinterpret_cast<uint32_t*>(p + 2 * st_bytes);
    s.tickets = s.ghist + 4 * kMaxBins;
    s.range = s.tickets + 4;
    return s;
}

uint32_t* sort_counters(void* ws, int64_t n_max, uint32_t* count) {
    *count = (uint32_t)(4 * kMaxBins + 6);
    return sort_ws(ws, n_max).ghist;
}

size_t radix_ws_bytes(int64_t n_max) {
    const int64_t nb = std::max<int64_t>(1, (n_max + kOsTile - 1) / kOsTile);
    return 2 * align_up(8 * (size_t)kMaxBins * (size_t)nb) + align_up(4 * (4 * (size_t)kMaxBins + 6));
}

// Digit histograms of every pass over the live keys (global atomics of each
// workgroup's nonzero LDS bins) and a zeroed state row per live tile for the
// first pass.  Each bin has LDS copies, lane l adding to copy l % copies,
// so lanes of a wave that share a digit (the high digits of depth keys take
// few values) collide at most 64 / copies ways.  DEPTH: digits of the keys
// relative to the depth range.
template <int RB, bool DEPTH, typename KT = uint32_t, int IT = kOsItems>
__global__ __launch_bounds__(kOsThreads) void k_os_hist(const KT* keys, int64_t n_max,
                                                        const unsigned long long* n_dev, int nbits, uint32_t* ghist,
                                                        uint64_t* status0, const uint32_t* range) {
    constexpr int KB = 1 << RB;
    constexpr int TILE = IT * kOsThreads;
    constexpr int kCopies = 8 >> (RB - 8);
    __shared__ uint32_t h[4 * KB * kCopies];
    for (int i = threadIdx.x; i < 4 * KB * kCopies; i += kOsThreads) h[i] = 0;
    __syncthreads();
    const uint32_t copy = threadIdx.x % kCopies;
    const int64_t n = live_count(n_max, n_dev);
    const int64_t nb = (n + TILE - 1) / TILE;
    int passes = (nbits + RB - 1) / RB;
    DepthRange dr{};
    if constexpr (DEPTH) {
        dr = depth_range(range);
        passes = depth_passes(dr);          // digits above the range are all zero: not counted
    }
    for (int64_t t = blockIdx.x; t < nb; t += gridDim.x) {
        if (threadIdx.x < KB) status0[t * KB + threadIdx.x] = 0ull;
        uint32_t k_[IT];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int64_t j = t * TILE + (int64_t)i * kOsThreads + threadIdx.x;
            k_[i] = j < n ? (uint32_t)keys[j] : 0u;
            if constexpr (DEPTH) k_[i] = depth_rel(k_[i], dr);
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int64_t j = t * TILE + (int64_t)i * kOsThreads + threadIdx.x;
            if (j < n)
                for (int p = 0; p < passes; ++p) {
                    const uint32_t d = (k_[i] >> (p * RB)) & pass_mask<RB>(nbits, p);
                    atomicAdd(&h[(p * KB + d) * kCopies + copy], 1u);
                }
        }
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        for (int b = threadIdx.x; b < KB; b += kOsThreads) {
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < kCopies; ++q) c += h[(p * KB + b) * kCopies + q];
            if (c) atomicAdd(&ghist[p * kMaxBins + b], c);     // rows laid out for the widest digit
        }
}

// One pass.  Wave w of the workgroup owns keys [64 IT w, 64 IT (w + 1)) of
// the tile (IT keys per lane) and walks them 64 at a time; ranks are computed in that item
// order (wave, step, lane), which keeps the sort stable: for each step the
// lanes OR their bit into an LDS mask per (wave, digit), read it back (the
// lanes sharing their digit), and the lowest of them advances the wave's
// count of the digit and clears the mask.  The keys then go to LDS in
// block-local digit order and out linearly, so each digit's run goes to
// consecutive global addresses; the values (and a payload word, if any)
// follow through the same LDS buffer.  Threads 0..bins-1 own one digit each
// for the counts and the look-back.
//
// MODE 0: plain.  1 (last pass): also gathers each value's tile rectangle
// from g.rect_in.  2: carries g.pay (pay_in -> pay_out).  3 (last pass):
// unpacks the payload (x0 | y0 << 8 | x1 << 16 | y1 << 24) into the
// rectangle and its tile count.  4: a pass of the depth sort (dio): exits if
// the depth range does not need it, picks its buffers so that the last
// pass the range needs writes the final ones, carries the payload, or
// unpacks it as in mode 3 when it is that last pass; the first pass makes
// the keys relative to the range.
constexpr int kPassPlain = 0, kPassGather = 1, kPassCarry = 2, kPassUnpack = 3, kPassDepth = 4;

struct DepthIO {
    const uint32_t* keys;       // raw depth keys
    const uint32_t* pay;        // packed rectangles
    uint32_t* kb[2];
    uint32_t* vb[2];
    uint32_t* pb[2];
    const uint32_t* range;
    int pass;
};

template <int MODE, int RB, typename KT = uint32_t, int IT = kOsItems>
__global__ __launch_bounds__(kOsThreads) void k_os_pass(const KT* keys_in, const uint32_t* vals_in,
                                                        KT* keys_out, uint32_t* vals_out, int64_t n_max,
                                                        const unsigned long long* n_dev, int shift, uint32_t mask,
                                                        const uint32_t* ghist, uint64_t* status,
                                                        uint64_t* status_next, uint32_t* ticket, SortGather g,
                                                        const uint32_t* pay_in, uint32_t* pay_out, DepthIO dio) {
    constexpr int KB = 1 << RB;
    constexpr int TILE = IT * kOsThreads;
    constexpr bool PAY = MODE == kPassCarry || MODE == kPassUnpack || MODE == kPassDepth;
    bool fin = MODE == kPassGather || MODE == kPassUnpack;    // writes the final rectangles
    DepthRange dr{};
    if constexpr (MODE == kPassDepth) {
        dr = depth_range(dio.range);
        const int L = depth_passes(dr);
        if (dio.pass >= L) return;                            // the range is covered already
        fin = dio.pass == L - 1;
        const int o = (L - 1 - dio.pass) & 1 ? 0 : 1;         // the last live pass writes buffer 1
        keys_in = dio.pass == 0 ? dio.keys : dio.kb[o ^ 1];
        vals_in = dio.pass == 0 ? nullptr : dio.vb[o ^ 1];
        pay_in = dio.pass == 0 ? dio.pay : dio.pb[o ^ 1];
        keys_out = fin ? nullptr : dio.kb[o];
        vals_out = dio.vb[o];
        pay_out = dio.pb[o];
        if (fin) status_next = nullptr;
    }
    __shared__ uint32_t cnt[kOsWaves][KB];
    // The peer masks are needed only while ranking, the staging buffer only
    // after it (two barriers later): they share the same LDS.
    __shared__ __align__(16) uint32_t s_buf[TILE];
    static_assert(sizeof(unsigned long long) * kOsWaves * KB <= sizeof(uint32_t) * TILE, "peer masks");
    unsigned long long (*s_peer)[KB] = reinterpret_cast<unsigned long long (*)[KB]>(s_buf);
    __shared__ uint32_t s_goff[KB];
    __shared__ uint32_t s_wave[kOsWaves];
    __shared__ uint32_t s_ticket;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_ticket = atomicAdd(ticket, 1u);
    for (int i = threadIdx.x; i < kOsWaves * KB; i += kOsThreads) {
        (&cnt[0][0])[i] = 0;
        (&s_peer[0][0])[i] = 0ull;
    }
    __syncthreads();
    const int64_t b = s_ticket;
    const int64_t n = live_count(n_max, n_dev);
    const int64_t blk0 = b * TILE;
    if (blk0 >= n) return;
    const bool dig = threadIdx.x < KB;
    const uint32_t d = dig ? threadIdx.x : 0u;
    if (status_next && dig) status_next[b * KB + d] = 0ull;
    const int64_t base = blk0 + (int64_t)w * (IT * 64);
    uint32_t k_[IT], v_[IT], p_[PAY ? IT : 1];
    uint32_t lp[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int64_t j = base + i * 64 + lane;
        k_[i] = j < n ? (uint32_t)keys_in[j] : 0u;
        if constexpr (MODE == kPassDepth)
            if (dio.pass == 0) k_[i] = depth_rel(k_[i], dr);
    }
    const unsigned long long bit = 1ull << lane;
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const bool live = base + i * 64 + lane < n;
        const uint32_t dd = (k_[i] >> shift) & mask;
        lp[i] = 0xffffffffu;
        if (live) atomicOr(&s_peer[w][dd], bit);
        wave_sync();
        if (live) {
            const uint64_t peers = s_peer[w][dd];
            const uint32_t below = popc_below(peers);
            const uint32_t run = cnt[w][dd];
            lp[i] = run + below;
            wave_sync();
            if (below == 0) {
                cnt[w][dd] = run + (uint32_t)__popcll(peers);
                s_peer[w][dd] = 0ull;
            }
        }
        wave_sync();
    }
    __syncthreads();
    uint32_t tot = 0, wb[kOsWaves];
#pragma unroll
    for (int i = 0; i < kOsWaves; ++i) { wb[i] = tot; tot += dig ? cnt[i][d] : 0u; }
    uint64_t* mine = status + b * KB + d;
    if (dig) status_put(mine, (b == 0 ? kStInc : (kStAgg | ((uint64_t)b << 32))) | (uint64_t)tot);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int64_t j = base + i * 64 + lane;
        v_[i] = j < n ? (vals_in ? vals_in[j] : (uint32_t)j) : 0u;
        if constexpr (PAY) p_[i] = j < n ? pay_in[j] : 0u;
    }
    const uint32_t gstart = os_scan(dig ? ghist[d] : 0u, s_wave);
    const uint32_t dstart = os_scan(tot, s_wave);
    if (dig)
        for (int i = 0; i < kOsWaves; ++i) cnt[i][d] = dstart + wb[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i)
        if (lp[i] != 0xffffffffu) {
            lp[i] += cnt[w][(k_[i] >> shift) & mask];
            s_buf[lp[i]] = k_[i];
        }
    uint32_t excl = 0;
    if (dig && b > 0) {
        int64_t k = b - 1;
        uint32_t spins = 0;
        for (;;) {
            const uint64_t s = status_get(status + k * KB + d);
            const uint64_t f = s >> 62;
            if (f == 0) {
                if (++spins >= kSpinLimit) { atomicAdd(&g_sort_stalls, 1u); break; }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += (uint32_t)s;
            if (f == 2) break;
            k = (int64_t)((s >> 32) & 0x3fffffffull) - 1;
            status_put(mine, kStAgg | ((uint64_t)(k + 1) << 32) | (uint64_t)(excl + tot));
        }
        status_put(mine, kStInc | (uint64_t)(excl + tot));
    }
    if (dig) s_goff[d] = gstart + excl - dstart;
    __syncthreads();
    const int m = (int)(n - blk0 < TILE ? n - blk0 : TILE);
    uint32_t pos[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int q = i * kOsThreads + (int)threadIdx.x;
        pos[i] = 0xffffffffu;
        if (q < m) {
            const uint32_t key = s_buf[q];
            pos[i] = s_goff[(key >> shift) & mask] + (uint32_t)q;
            if (keys_out && (int64_t)pos[i] < n) keys_out[pos[i]] = (KT)key;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i)
        if (lp[i] != 0xffffffffu) s_buf[lp[i]] = v_[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int q = i * kOsThreads + (int)threadIdx.x;
        if (q < m && (int64_t)pos[i] < n) {
            const uint32_t v = s_buf[q];
            vals_out[pos[i]] = v;
            if constexpr (MODE == kPassGather) {
                const uint2 tr = g.rect_in[v];
                const uint32_t x0 = tr.x & 0xffffu, y0 = tr.x >> 16, x1 = tr.y & 0xffffu, y1 = tr.y >> 16;
                g.rect_out[pos[i]] = tr;
                g.cnt_out[pos[i]] = (x1 > x0 && y1 > y0) ? (x1 - x0) * (y1 - y0) : 0u;
            }
        }
    }
    if constexpr (PAY) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i)
            if (lp[i] != 0xffffffffu) s_buf[lp[i]] = p_[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int q = i * kOsThreads + (int)threadIdx.x;
            if (q < m && (int64_t)pos[i] < n) {
                const uint32_t pw = s_buf[q];
                if (!fin) {
                    pay_out[pos[i]] = pw;
                } else {
                    const uint32_t x0 = pw & 0xffu, y0 = (pw >> 8) & 0xffu, x1 = (pw >> 16) & 0xffu, y1 = pw >> 24;
                    g.rect_out[pos[i]] = make_uint2(x0 | (y0 << 16), x1 | (y1 << 16));
                    g.cnt_out[pos[i]] = (x1 > x0 && y1 > y0) ? (x1 - x0) * (y1 - y0) : 0u;
                }
            }
        }
    }
}

template <typename KT>
int radix_sort_impl(const KT* kin, const uint32_t* vin, KT* kbuf[2], uint32_t* vbuf[2], int64_t n_max,
                    const unsigned long long* n_dev, int nbits, void* ws, hipStream_t st, hipError_t* err,
                    const SortGather* last, bool zeroed) {
    *err = hipSuccess;
    constexpr int IT = os_items<KT>();
    constexpr int64_t TILE = IT * kOsThreads;
    const int passes = (nbits + kRadixBits - 1) / kRadixBits;
    const int final_buf = passes > 0 ? (passes - 1) & 1 : 0;
    const int64_t nblocks = (n_max + TILE - 1) / TILE;
    if (nblocks == 0 || nbits <= 0) return final_buf;
    if (passes > 4) { *err = hipErrorInvalidValue; return final_buf; }
    const SortWs s = sort_ws(ws, n_max);
    if (!zeroed) *err = fill_u32(s.ghist, 0u, 4 * kMaxBins + 6, st);
    if (*err != hipSuccess) return final_buf;
    const unsigned hb = (unsigned)std::min<int64_t>(nblocks, kOsHistBlocks);
    hipLaunchKernelGGL((k_os_hist<kRadixBits, false, KT, IT>), dim3(hb), dim3(kOsThreads), 0, st, kin, n_max, n_dev,
                       nbits, s.ghist, s.status[0], nullptr);
    const KT* ksrc = kin;
    const uint32_t* vsrc = vin;
    const DepthIO none{};
    for (int p = 0; p < passes; ++p) {
        const int out = p & 1;
        const bool fin = p + 1 == passes;
        SortGather g{};
        const uint32_t* pin = nullptr;
        uint32_t* pout = nullptr;
        auto kern = k_os_pass<kPassPlain, kRadixBits, KT, IT>;
        if constexpr (sizeof(KT) == 4) {
            if (last && last->pay_in) {       // payload carried through every pass
                g = *last;
                pin = p == 0 ? last->pay_in : last->pay_buf[(p - 1) & 1];
                pout = last->pay_buf[p & 1];
                kern = fin ? k_os_pass<kPassUnpack, kRadixBits> : k_os_pass<kPassCarry, kRadixBits>;
            } else if (fin && last && last->rect_in) {
                g = *last;
                kern = k_os_pass<kPassGather, kRadixBits>;
            }
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(kOsThreads), 0, st, ksrc, vsrc,
                           fin && last && last->drop_keys ? nullptr : kbuf[out],
                           vbuf[out], n_max, n_dev, p * kRadixBits,
                           (uint32_t)((1ull << std::min(kRadixBits, nbits - p * kRadixBits)) - 1ull),
                           s.ghist + p * kMaxBins, s.status[p & 1], p + 1 < passes ? s.status[(p + 1) & 1] : nullptr,
                           s.tickets + p, g, pin, pout, none);
        ksrc = kbuf[out];
        vsrc = vbuf[out];
    }
    *err = hipGetLastError();
    return final_buf;
}

int radix_sort_pairs(const uint32_t* kin, const uint32_t* vin, uint32_t* kbuf[2], uint32_t* vbuf[2], int64_t n_max,
                     const unsigned long long* n_dev, int nbits, void* ws, hipStream_t st, hipError_t* err,
                     const SortGather* last, bool zeroed) {
    return radix_sort_impl<uint32_t>(kin, vin, kbuf, vbuf, n_max, n_dev, nbits, ws, st, err, last, zeroed);
}

int radix_sort_pairs16(const uint16_t* kin, const uint32_t* vin, uint16_t* kbuf[2], uint32_t* vbuf[2], int64_t n_max,
                       const unsigned long long* n_dev, int nbits, void* ws, hipStream_t st, hipError_t* err,
                       bool zeroed) {
    if (nbits > 16) { *err = hipErrorInvalidValue; return 0; }
    return radix_sort_impl<uint16_t>(kin, vin, kbuf, vbuf, n_max, n_dev, nbits, ws, st, err, nullptr, zeroed);
}

// The depth sort of the records (31-bit keys, +inf for culled records) with
// the packed-rectangle payload: the result is in kbuf/vbuf[1] and g's
// rectangle and count arrays whatever the number of passes the range takes.
int radix_sort_depth(const uint32_t* kin, const uint32_t* krange, int64_t n_part, uint32_t* kbuf[2], uint32_t* vbuf[2],
                     int64_t n, void* ws, hipStream_t st, hipError_t* err, const SortGather& g, bool zeroed) {
    *err = hipSuccess;
    const int64_t nblocks = (n + kOsTile - 1) / kOsTile;
    if (nblocks == 0) return 1;
    const SortWs s = sort_ws(ws, n);
    if (!zeroed) *err = fill_u32(s.ghist, 0u, 4 * kMaxBins + 6, st);
    if (*err != hipSuccess) return 1;
    const unsigned hb = (unsigned)std::min<int64_t>(nblocks, kOsHistBlocks);
    const unsigned rb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_part + 255) / 256, 256));
    hipLaunchKernelGGL(k_key_range, dim3(rb), dim3(256), 0, st, reinterpret_cast<const uint2*>(krange), n_part,
                       s.range);
    hipLaunchKernelGGL((k_os_hist<kDepthBits, true>), dim3(hb), dim3(kOsThreads), 0, st, kin, n, nullptr, 31,
                       s.ghist, s.status[0], s.range);
    constexpr int kPasses = (31 + kDepthBits - 1) / kDepthBits;
    for (int p = 0; p < kPasses; ++p) {
        DepthIO io{kin, g.pay_in, {kbuf[0], kbuf[1]}, {vbuf[0], vbuf[1]}, {g.pay_buf[0], g.pay_buf[1]}, s.range, p};
        hipLaunchKernelGGL((k_os_pass<kPassDepth, kDepthBits, uint32_t>), dim3((unsigned)nblocks), dim3(kOsThreads), 0, st,
                           nullptr, nullptr, nullptr, nullptr, n, nullptr, p * kDepthBits, (uint32_t)(kMaxBins - 1),
                           s.ghist + p * kMaxBins, s.status[p & 1], p + 1 < kPasses ? s.status[(p + 1) & 1] : nullptr,
                           s.tickets + p, g, nullptr, nullptr, io);
    }
    *err = hipGetLastError();
    return 1;
}

int64_t resident_blocks(const void* kernel, int block) {
    struct Entry { int dev, block; const void* kernel; int64_t n; };
    static Entry table[64];
    static int used = 0;
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < used; ++i)
        if (table[i].dev == dev && table[i].kernel == kernel && table[i].block == block) return table[i].n;
    int ncu = 0, per = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess || ncu <= 0)
        return 0;
    const int64_t n = (int64_t)ncu * (per > 0 ? per : 1);
    if (used < 64) table[used++] = Entry{dev, block, kernel, n};
    return n;
}

uint32_t sort_stalls() {
    uint32_t v = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_sort_stalls), sizeof(v), 0, hipMemcpyDeviceToHost) != hipSuccess)
        return 0xffffffffu;
    return v;
}

// ----------------------------------------------------------- tile ranges
// ranges[t] = [lower_bound(t), lower_bound(t+1)) over the sorted tile keys.
template <typename KT>
__global__ void k_tile_ranges(const KT* sorted, const unsigned long long* n_dev, int64_t n_max,
                              int64_t n_tiles, uint32_t* ranges) {
    // thread t finds lower_bound(t), the start of tile t and the end of
    // tile t - 1 (thread n_tiles finds the end of the last tile)
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n_tiles) return;
    const int64_t n = live_count(n_max, n_dev);
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)sorted[mid] < t) lo = mid + 1; else hi = mid;
    }
    if (t < n_tiles) ranges[2 * t] = (uint32_t)lo;
    if (t > 0) ranges[2 * (t - 1) + 1] = (uint32_t)lo;
}

// 8-bit sort key of each tile for the heavy-first order: 255 - q(length),
// q exact below 128 and log-scaled above (16 steps per doubling, 255 from
// 2^15 on), non-decreasing in the length, so one stable 8-bit pass orders
// the tiles longest first (ties and lengths sharing a step by tile index).
__global__ void k_tile_len_keys(const uint32_t* ranges, int64_t n_tiles, uint32_t* key) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    uint32_t q = len;
    if (len >= 128u) {
        const int b = 32 - __clz((int)len);      // bit length, 8..32
        q = 128u + 16u * (uint32_t)(b - 8) + ((len >> (b - 5)) & 15u);
        if (q > 255u) q = 255u;
    }
    key[t] = 255u - q;
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
    hipLaunchKernelGGL(k_tile_ranges<uint32_t>, dim3((unsigned)((n_tiles + 1 + 255) / 256)), dim3(256), 0, st,
                       sorted_tile, n_dev, n_max, n_tiles, ranges);
    return hipGetLastError();
}

hipError_t tile_ranges16(const uint16_t* sorted_tile, const unsigned long long* n_dev, int64_t n_max,
                         int64_t n_tiles, uint32_t* ranges, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_ranges<uint16_t>, dim3((unsigned)((n_tiles + 1 + 255) / 256)), dim3(256), 0, st,
                       sorted_tile, n_dev, n_max, n_tiles, ranges);
    return hipGetLastError();
}

}  // namespace cgs
