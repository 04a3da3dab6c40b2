// Metropolis-Hastings split and merge moves on a codebook (the split and
// merge transitions of the proposal mixture, Sec. 4.4 and App. A.1), batched
// for the GPU: B independent proposals per step, one thread each, from
// Philox streams (counter 16 b + j, tag 0x20000 split / 0x20001 merge).
//
// Split proposal b: Gaussian g = choice(w0, N), offset u ~ N(0, eps_split^2 I)
// over the row (normals of counters j = 1..15), accepted iff
// log U < min(0, -lambda - log q_sm(|u|^2)), U = uniform24(w1),
// log q_sm(s) = -s/2 (1/eps_split^2 - 1/eps_merge^2).  A Gaussian named by
// several accepted proposals splits once (the lowest b: integer atomicMin, so
// the outcome does not depend on scheduling); the survivors in b order take
// new rows K, K+1, ... (exclusive scan of their flags) while rows remain: new
// row = C[idx[g]] + u, idx[g] = new row.
//
// Merge proposal b: rows c = choice(w0, K), c' = choice(w1, K-1) (+1 if >= c),
// accepted iff log U < -|c - c'|^2 / (2 eps_merge^2) + min(0, lambda +
// log q_sm(|c - c'|^2)), U = uniform24(w2): thinning uniform pairs by the
// Gaussian density selects pairs distributed as q_merge, and the second term
// is the paper's acceptance.  A row joins at most one merge per step (a
// proposal whose rows were named by an earlier accepted proposal is
// withdrawn, again by atomicMin).  The Gaussians of c' move to c (c keeps its
// value); the freed rows below K' = K - merges take the surviving rows at or
// above K' in ascending order, so live rows stay 0 .. K'-1.
//
// The live row count K stays on the device (graph-capturable, no host sync).
#include <algorithm>

#include "cgs_internal.h"
#include "philox.h"

namespace cgs {

constexpr uint32_t kSplitTag = 0x20000u, kMergeTag = 0x20001u, kMixTag = 0x20002u;
constexpr uint32_t kNone = 0xffffffffu;

__device__ inline uint4 mh_words(const MhArgs& a, int64_t b, int j, uint32_t tag) {
    const uint64_t i = 16u * (uint64_t)b + (uint64_t)j;
    return philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), tag, a.step), (uint32_t)a.seed,
                         (uint32_t)(a.seed >> 32));
}

__device__ inline float log_q_sm(const MhArgs& a, float s) { return -0.5f * s * (a.inv_s2 - a.inv_m2); }

__device__ inline void put_row_value(const MhArgs& a, int64_t row, int64_t d, float v) {
    a.rows[row * a.ld + d] = v;
    if (a.mirror) a.mirror[row * a.mirror_ld + d] = f32_to_bf16_rne(v);
}

__global__ void k_mh_fill(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ split
__global__ __launch_bounds__(256) void k_split_propose(MhArgs a, uint32_t* mark, uint32_t* acc, uint32_t* gsel,
                                                       float* u) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const uint4 w = mh_words(a, b, 0, kSplitTag);
    const uint32_t g = choice32(w.x, (uint32_t)a.n);
    float s = 0.f;
    float* ub = u + b * a.D;
    for (int j = 1; 4 * (j - 1) < a.D; ++j) {
        const uint4 wj = mh_words(a, b, j, kSplitTag);
        float z[4];
        box_muller_pair(wj.x, wj.y, z[0], z[1]);
        box_muller_pair(wj.z, wj.w, z[2], z[3]);
        for (int k = 0; k < 4 && 4 * (j - 1) + k < a.D; ++k) {
            const float v = a.eps_split * z[k];
            ub[4 * (j - 1) + k] = v;
            s = fmaf(v, v, s);
        }
    }
    const float log_a = fminf(0.f, -a.lambda - log_q_sm(a, s));
    const bool ok = a.n > 0 && logf(uniform24(w.y)) < log_a;
    acc[b] = ok ? 1u : 0u;
    gsel[b] = g;
    if (ok) atomicMin(&mark[g], (uint32_t)b);
}

__global__ __launch_bounds__(256) void k_split_valid(MhArgs a, const uint32_t* mark, const uint32_t* acc,
                                                     const uint32_t* gsel, uint32_t* valid) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    valid[b] = (acc[b] && mark[gsel[b]] == (uint32_t)b) ? 1u : 0u;
}

// one thread per proposal: it reads idx[g] before writing it
__global__ __launch_bounds__(256) void k_split_commit(MhArgs a, const uint32_t* valid, const uint32_t* rank,
                                                      const uint32_t* gsel, const float* u) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B || !valid[b]) return;
    const int64_t K = *a.d_rows;
    const int64_t row = K + (int64_t)rank[b];
    if (row >= a.K_max) return;
    const uint32_t g = gsel[b];
    const int64_t src = a.idx[g];
    for (int64_t d = 0; d < a.D; ++d) put_row_value(a, row, d, a.rows[src * a.ld + d] + u[b * a.D + d]);
    a.idx[g] = (int32_t)row;
}

__global__ void k_split_finish(MhArgs a, const unsigned long long* n_valid) {
    const int64_t K = *a.d_rows;
    const int64_t K2 = K + (int64_t)*n_valid;
    *a.d_rows = K2 < a.K_max ? K2 : a.K_max;
}

// ------------------------------------------------------------------ merge
__global__ __launch_bounds__(256) void k_merge_propose(MhArgs a, uint32_t* mark, uint32_t* acc, uint32_t* c0,
                                                       uint32_t* c1) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const int64_t K = *a.d_rows;
    acc[b] = 0u;
    if (K < 2) return;
    const uint4 w = mh_words(a, b, 0, kMergeTag);
    const uint32_t c = choice32(w.x, (uint32_t)K);
    uint32_t c2 = choice32(w.y, (uint32_t)(K - 1));
    c2 += c2 >= c ? 1u : 0u;
    float s = 0.f;
    for (int64_t d = 0; d < a.D; ++d) {
        const float e = a.rows[(int64_t)c * a.ld + d] - a.rows[(int64_t)c2 * a.ld + d];
        s = fmaf(e, e, s);
    }
    const float t = -0.5f * s * a.inv_m2 + fminf(0.f, a.lambda + log_q_sm(a, s));
    const bool ok = logf(uniform24(w.z)) < t;
    c0[b] = c;
    c1[b] = c2;
    if (ok) {
        acc[b] = 1u;
        atomicMin(&mark[c], (uint32_t)b);
        atomicMin(&mark[c2], (uint32_t)b);
    }
}

__global__ __launch_bounds__(256) void k_merge_valid(MhArgs a, const uint32_t* mark, const uint32_t* acc,
                                                     const uint32_t* c0, const uint32_t* c1, uint32_t* valid) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    valid[b] = (acc[b] && mark[c0[b]] == (uint32_t)b && mark[c1[b]] == (uint32_t)b) ? 1u : 0u;
}

// Per row r < K: freed (the c' of a surviving merge) and, for the
// compaction scan, flag = freed for r < K', not freed for r >= K'.
__global__ __launch_bounds__(256) void k_merge_rows(MhArgs a, const uint32_t* mark, const uint32_t* valid,
                                                    const uint32_t* c0, const uint32_t* c1,
                                                    const unsigned long long* n_merges, uint32_t* partner,
                                                    uint32_t* flag) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.K_max) return;
    const int64_t K = *a.d_rows;
    const int64_t K2 = K - (int64_t)*n_merges;
    uint32_t p = kNone, f = 0u;
    if (r < K) {
        const uint32_t m = mark[r];
        const bool freed = m != kNone && valid[m] && c1[m] == (uint32_t)r;
        if (freed) p = c0[m];
        f = r < K2 ? (freed ? 1u : 0u) : (freed ? 0u : 1u);
    }
    partner[r] = p;
    flag[r] = f;
}

// hole_of[rank] = the rank-th freed row below K'
__global__ __launch_bounds__(256) void k_merge_holes(MhArgs a, const unsigned long long* n_merges,
                                                     const uint32_t* flag, const uint32_t* scan, uint32_t* hole_of) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t K2 = *a.d_rows - (int64_t)*n_merges;
    if (r >= K2) return;
    if (flag[r]) hole_of[scan[r]] = (uint32_t)r;
}

// final[r] = new index of the row Gaussians on r end up on; movers copy
// their values into their hole
__global__ __launch_bounds__(256) void k_merge_final(MhArgs a, const unsigned long long* n_merges,
                                                     const uint32_t* partner, const uint32_t* flag,
                                                     const uint32_t* scan, const uint32_t* hole_of, uint32_t* fin) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t K = *a.d_rows;
    if (r >= K) return;
    const int64_t K2 = K - (int64_t)*n_merges;
    const uint32_t base = K2 < K ? scan[K2] : 0u;     // holes below K'
    auto moved = [&](int64_t x) -> uint32_t {
        if (x >= K2 && flag[x]) return hole_of[scan[x] - base];
        return (uint32_t)x;
    };
    const int64_t keep = partner[r] != kNone ? (int64_t)partner[r] : r;
    fin[r] = moved(keep);
    if (r >= K2 && flag[r]) {
        const int64_t h = hole_of[scan[r] - base];
        for (int64_t d = 0; d < a.D; ++d) put_row_value(a, h, d, a.rows[r * a.ld + d]);
    }
}

__global__ __launch_bounds__(256) void k_merge_remap(MhArgs a, const uint32_t* fin) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    a.idx[g] = (int32_t)fin[a.idx[g]];
}

__global__ void k_merge_finish(MhArgs a, const unsigned long long* n_merges) {
    *a.d_rows = *a.d_rows - (int64_t)*n_merges;
}

// ------------------------------------------------------------------ host
namespace {
inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }
}

size_t mh_workspace(int64_t B, int64_t D, int64_t K_max, int64_t n, MhWs* w, char* base) {
    size_t o = 0;
    auto take = [&](size_t bytes) { char* p = base ? base + o : nullptr; o = (o + bytes + 255) & ~(size_t)255; return p; };
    const int64_t nm = std::max(n, K_max);
    const int64_t big = std::max(B, K_max);
    MhWs t;
    t.mark = (uint32_t*)take(4 * (size_t)nm);
    t.acc = (uint32_t*)take(4 * (size_t)B);
    t.s0 = (uint32_t*)take(4 * (size_t)B);
    t.s1 = (uint32_t*)take(4 * (size_t)B);
    t.valid = (uint32_t*)take(4 * (size_t)B);
    t.rank = (uint32_t*)take(4 * (size_t)B);
    t.partner = (uint32_t*)take(4 * (size_t)K_max);
    t.flag = (uint32_t*)take(4 * (size_t)K_max);
    t.scan = (uint32_t*)take(4 * (size_t)K_max);
    t.hole_of = (uint32_t*)take(4 * (size_t)K_max);
    t.fin = (uint32_t*)take(4 * (size_t)K_max);
    t.u = (float*)take(4 * (size_t)B * (size_t)D);
    t.tot = (unsigned long long*)take(16);
    t.bsum = (unsigned long long*)take(8 * (size_t)((big + kSortTile - 1) / kSortTile + 2));
    if (w) *w = t;
    return o;
}

hipError_t mh_split(const MhArgs& a, const MhWs& w, hipStream_t st) {
    hipLaunchKernelGGL(k_mh_fill, dim3(nblk(a.n)), dim3(256), 0, st, w.mark, a.n, kNone);
    hipLaunchKernelGGL(k_split_propose, dim3(nblk(a.B)), dim3(256), 0, st, a, w.mark, w.acc, w.s0, w.u);
    hipLaunchKernelGGL(k_split_valid, dim3(nblk(a.B)), dim3(256), 0, st, a, w.mark, w.acc, w.s0, w.valid);
    hipError_t e = scan_u32(w.valid, nullptr, a.B, w.rank, w.tot, w.bsum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_commit, dim3(nblk(a.B)), dim3(256), 0, st, a, w.valid, w.rank, w.s0, w.u);
    hipLaunchKernelGGL(k_split_finish, dim3(1), dim3(1), 0, st, a, w.tot);
    return hipGetLastError();
}

hipError_t mh_merge(const MhArgs& a, const MhWs& w, hipStream_t st) {
    hipLaunchKernelGGL(k_mh_fill, dim3(nblk(a.K_max)), dim3(256), 0, st, w.mark, a.K_max, kNone);
    hipLaunchKernelGGL(k_merge_propose, dim3(nblk(a.B)), dim3(256), 0, st, a, w.mark, w.acc, w.s0, w.s1);
    hipLaunchKernelGGL(k_merge_valid, dim3(nblk(a.B)), dim3(256), 0, st, a, w.mark, w.acc, w.s0, w.s1, w.valid);
    hipError_t e = scan_u32(w.valid, nullptr, a.B, w.rank, w.tot, w.bsum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_rows, dim3(nblk(a.K_max)), dim3(256), 0, st, a, w.mark, w.valid, w.s0, w.s1, w.tot,
                       w.partner, w.flag);
    e = scan_u32(w.flag, nullptr, a.K_max, w.scan, w.tot + 1, w.bsum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_holes, dim3(nblk(a.K_max)), dim3(256), 0, st, a, w.tot, w.flag, w.scan, w.hole_of);
    hipLaunchKernelGGL(k_merge_final, dim3(nblk(a.K_max)), dim3(256), 0, st, a, w.tot, w.partner, w.flag, w.scan,
                       w.hole_of, w.fin);
    hipLaunchKernelGGL(k_merge_remap, dim3(nblk(a.n)), dim3(256), 0, st, a, w.fin);
    hipLaunchKernelGGL(k_merge_finish, dim3(1), dim3(1), 0, st, a, w.tot);
    return hipGetLastError();
}

int mh_transition_host(uint64_t seed, uint32_t step) {
    const uint4 w = philox4x32_10(make_uint4(0u, 0u, kMixTag, step), (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u = ((double)(w.x >> 8) + 0.5) * 5.9604644775390625e-08;
    return u < 0.98 ? 0 : (u < 0.99 ? 1 : 2);
}

}  // namespace cgs
