// Training-step pieces around the render: the reconstruction loss of Eq. 4,
// L = (1 - lambda) L1 + lambda (1 - mean SSIM), with its gradient with respect
// to the rendered image, and the standalone noise generator of the SGLD
// update (the update itself is fused into the backward's epilogues).
//
// SSIM (Wang et al. 2004) per pixel and channel from local statistics under
// an 11x11 Gaussian window (sigma 1.5, normalised, separable), "same"-size
// with zero padding, C1 = 0.01^2, C2 = 0.03^2:
//   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)),
//   mx = w*x, sxx = w*(x x) - mx^2, sxy = w*(x y) - mx my.
// With A1, A2, B1, B2 the four factors (B1, B2 > 0; A2 = 2 sxy + C2 may
// vanish, so nothing divides by it), S depends on the image x through
//   dS/dmx  = 2 [my (A2 - A1) - mx S (B2 - B1)] / (B1 B2),
//   dS/dmxx = -S / B2,   dS/dmxy = 2 A1 / (B1 B2)   (mxx = w*(x x), mxy = w*(x y)),
// and the window is symmetric, so
//   d(sum_q S(q))/dx(p) = w*(dS/dmx)(p) + 2 x(p) w*(dS/dmxx)(p) + y(p) w*(dS/dmxy)(p)
// with the partial maps taken as zero outside the image.  Only sxx + syy
// enters S, so the statistics pass blurs x^2 + y^2 as one map (four window
// sums per channel: x, y, x^2 + y^2, x y); its partial is dS/dmxx above.
//
// Two tiled passes per 16x16 pixel tile (256 threads, one pixel each): the
// statistics pass blurs the tile plus a 5-pixel halo of image and target,
// rows then columns (each blur thread loads its line -- a row straight from
// memory, a column from the row sums in LDS -- and slides its 11-tap window
// along it in registers, the taps added in the same order for every
// output), and writes the three partials per channel
// and the tile's L1 and SSIM sums; the gradient pass blurs the partial maps
// the same way and combines them with the image, the target and the L1 term.
// A last single-workgroup pass adds the tile sums in a fixed order in FP64.
#include "cgs_internal.h"
#include "philox.h"

namespace cgs {

namespace {

constexpr int kHalo = 5;
constexpr int kSpan = kTile + 2 * kHalo;   // 26
// normalised exp(-k^2 / (2 * 1.5^2)), k = -5..5, rounded to FP32
__constant__ float kWin[11] = {1.028380124e-03f, 7.598758209e-03f, 3.600077331e-02f, 1.093606874e-01f,
                               2.130055428e-01f, 2.660117149e-01f, 2.130055428e-01f, 1.093606874e-01f,
                               3.600077331e-02f, 7.598758209e-03f, 1.028380124e-03f};
constexpr float kC1 = 1e-4f;
constexpr float kC2 = 9e-4f;

}  // namespace

__device__ inline int loss_view_of(const LossViews& v, int64_t t) {
    int lo = 0, hi = v.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (v.tile_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_ssim_stats(LossViews lv, const float* __restrict__ image,
                                                    const float* __restrict__ target, float* __restrict__ part,
                                                    double* __restrict__ sums) {
    __shared__ float s_h[12][kSpan][kTile];
    __shared__ float s_m[12][kTile][kTile];
    __shared__ double s_red[2][4];
    const int64_t t = blockIdx.x;
    const int v = loss_view_of(lv, t);
    const int H = lv.H[v], W = lv.W[v];
    const int64_t lt = t - lv.tile_off[v];
    const int x0 = (int)(lt % lv.tiles_x[v]) * kTile, y0 = (int)(lt / lv.tiles_x[v]) * kTile;
    const float* img = image + 3 * lv.pix_off[v];
    const float* tgt = target + 3 * lv.pix_off[v];
    // rows: four window sums per (row, output column, channel) -- x, y,
    // x^2 + y^2 (only sxx + syy enters S) and x y; a thread takes eight
    // outputs of one row, loads its 18 values of image and target straight
    // from memory (all in flight at once, no staging buffer) and slides the
    // window in registers
    if (threadIdx.x < kSpan * 3 * 2) {
        const int r = threadIdx.x / 6, ch = (threadIdx.x / 2) % 3, c0 = 8 * (threadIdx.x & 1);
        const int gy = y0 - kHalo + r;
        const bool rin = gy >= 0 && gy < H;
        const int64_t ro = 3 * (int64_t)(rin ? gy : 0) * W + ch;
        float a[18], b[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const int gx = x0 - kHalo + c0 + k;
            const bool in = rin && gx >= 0 && gx < W;
            a[k] = in ? img[ro + 3 * gx] : 0.f;
            b[k] = in ? tgt[ro + 3 * gx] : 0.f;
        }
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            float hx = 0.f, hy = 0.f, hs = 0.f, hxy = 0.f;
#pragma unroll
            for (int k = 0; k < 11; ++k) {
                const float aa = a[o + k], bb = b[o + k], w = kWin[k];
                hx = fmaf(w, aa, hx);
                hy = fmaf(w, bb, hy);
                hs = fmaf(w, fmaf(aa, aa, bb * bb), hs);
                hxy = fmaf(w, aa * bb, hxy);
            }
            s_h[4 * ch + 0][r][c0 + o] = hx;
            s_h[4 * ch + 1][r][c0 + o] = hy;
            s_h[4 * ch + 2][r][c0 + o] = hs;
            s_h[4 * ch + 3][r][c0 + o] = hxy;
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    const int gx = x0 + tx, gy = y0 + ty;
    // columns: a thread takes one (quantity, column) and slides down it
    if (threadIdx.x < 12 * kTile) {
        const int l = threadIdx.x / kTile, c = threadIdx.x % kTile;
        float col[kSpan];
#pragma unroll
        for (int k = 0; k < kSpan; ++k) col[k] = s_h[l][k][c];
#pragma unroll
        for (int o = 0; o < kTile; ++o) {
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < 11; ++k) a = fmaf(kWin[k], col[o + k], a);
            s_m[l][o][c] = a;
        }
    }
    __syncthreads();
    double l1 = 0.0, ss = 0.0;
    if (gx < W && gy < H) {
        const int64_t p = lv.pix_off[v] + (int64_t)gy * W + gx;
        float* out = part + 9 * p;
        float cx[3], cy[3];     // this pixel's image and target values, for the L1 term
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) { cx[ch] = image[3 * p + ch]; cy[ch] = target[3 * p + ch]; }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float m[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) m[q] = s_m[4 * ch + q][ty][tx];
            const float mx = m[0], my = m[1];
            const float A1 = 2.f * mx * my + kC1;
            const float A2 = 2.f * (m[3] - mx * my) + kC2;
            const float B1 = mx * mx + my * my + kC1;
            const float B2 = ((m[2] - mx * mx) - my * my) + kC2;
            const float inv = 1.f / (B1 * B2);
            const float S = A1 * A2 * inv;
            out[3 * ch + 0] = 2.f * inv * (my * (A2 - A1) - mx * S * (B2 - B1));
            out[3 * ch + 1] = -S / B2;
            out[3 * ch + 2] = 2.f * A1 * inv;
            ss += (double)S;
            l1 += (double)fabsf(cx[ch] - cy[ch]);
        }
    }
    // tile sums: butterfly over each wave, then the four waves in order
    for (int d = 32; d >= 1; d >>= 1) {
        l1 += __shfl_xor(l1, d, 64);
        ss += __shfl_xor(ss, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_red[0][threadIdx.x >> 6] = l1;
        s_red[1][threadIdx.x >> 6] = ss;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sums[2 * t] = (s_red[0][0] + s_red[0][1]) + (s_red[0][2] + s_red[0][3]);
        sums[2 * t + 1] = (s_red[1][0] + s_red[1][1]) + (s_red[1][2] + s_red[1][3]);
    }
}

__global__ __launch_bounds__(256) void k_ssim_grad(LossViews lv, const float* __restrict__ image,
                                                   const float* __restrict__ target, const float* __restrict__ part,
                                                   float l1w, float ssw, float* __restrict__ grad) {
    __shared__ float s_h[9][kSpan][kTile];
    __shared__ float s_m[9][kTile][kTile];
    const int64_t t = blockIdx.x;
    const int v = loss_view_of(lv, t);
    const int H = lv.H[v], W = lv.W[v];
    const int64_t lt = t - lv.tile_off[v];
    const int x0 = (int)(lt % lv.tiles_x[v]) * kTile, y0 = (int)(lt / lv.tiles_x[v]) * kTile;
    const float* pp = part + 9 * lv.pix_off[v];
    // rows, then columns, each thread sliding an 11-tap window along one
    // line; a row thread loads its 26 values straight from the partial maps
    // (all loads in flight at once, no staging buffer)
    if (threadIdx.x < kSpan * 9) {
        const int r = threadIdx.x / 9, q = threadIdx.x % 9;
        const int gy = y0 - kHalo + r;
        const bool rin = gy >= 0 && gy < H;
        const float* src = pp + 9 * ((int64_t)(rin ? gy : 0) * W) + q;
        float row[kSpan];
#pragma unroll
        for (int k = 0; k < kSpan; ++k) {
            const int gx = x0 - kHalo + k;
            row[k] = rin && gx >= 0 && gx < W ? src[9 * gx] : 0.f;
        }
#pragma unroll
        for (int o = 0; o < kTile; ++o) {
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < 11; ++k) a = fmaf(kWin[k], row[o + k], a);
            s_h[q][r][o] = a;
        }
    }
    __syncthreads();
    if (threadIdx.x < 9 * kTile) {
        const int q = threadIdx.x / kTile, c = threadIdx.x % kTile;
        float col[kSpan];
#pragma unroll
        for (int k = 0; k < kSpan; ++k) col[k] = s_h[q][k][c];
#pragma unroll
        for (int o = 0; o < kTile; ++o) {
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < 11; ++k) a = fmaf(kWin[k], col[o + k], a);
            s_m[q][o][c] = a;
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    const int gx = x0 + tx, gy = y0 + ty;
    if (gx >= W || gy >= H) return;
    const int64_t p = lv.pix_off[v] + (int64_t)gy * W + gx;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float b[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) b[q] = s_m[3 * ch + q][ty][tx];
        const float x = image[3 * p + ch], y = target[3 * p + ch];
        const float d = x - y;
        const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        const float dS = b[0] + 2.f * x * b[1] + y * b[2];
        grad[3 * p + ch] = l1w * sg - ssw * dS;
    }
}

// loss = (1 - lambda) L1sum / n + lambda (1 - Ssum / n), sums in FP64 in a fixed
// order; each thread loads eight tile pairs at a time, then adds them in index order
__global__ __launch_bounds__(1024) void k_loss_final(const double* __restrict__ sums, int64_t nt, int64_t n,
                                                     float lambda, float* __restrict__ loss) {
    __shared__ double s[2][1024];
    double a = 0.0, b = 0.0;
    for (int64_t i0 = threadIdx.x; i0 < nt; i0 += 8 * 1024) {
        double ua[8], ub[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = i0 + (int64_t)k * 1024;
            ua[k] = i < nt ? sums[2 * i] : 0.0;
            ub[k] = i < nt ? sums[2 * i + 1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a += ua[k];
            b += ub[k];
        }
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    __syncthreads();
    for (int d = 512; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            s[0][threadIdx.x] += s[0][threadIdx.x + d];
            s[1][threadIdx.x] += s[1][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double inv = n > 0 ? 1.0 / (double)n : 0.0;
        *loss = (float)((1.0 - (double)lambda) * s[0][0] * inv + (double)lambda * (1.0 - s[1][0] * inv));
    }
}

hipError_t launch_loss_recon(const LossViews& lv, const float* image, const float* target, float lambda, float* grad,
                             float* loss, float* part, double* sums, hipStream_t st) {
    const int64_t nt = lv.tile_off[lv.n];
    int64_t n = 0;
    for (int v = 0; v < lv.n; ++v) n += 3 * (int64_t)lv.H[v] * lv.W[v];
    if (nt > 0) {
        hipLaunchKernelGGL(k_ssim_stats, dim3((unsigned)nt), dim3(256), 0, st, lv, image, target, part, sums);
        const float inv = (float)(1.0 / (double)n);
        hipLaunchKernelGGL(k_ssim_grad, dim3((unsigned)nt), dim3(256), 0, st, lv, image, target, part,
                           (1.f - lambda) * inv, lambda * inv, grad);
    }
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, st, sums, nt, n, lambda, loss);
    return hipGetLastError();
}

// ------------------------------------------------------------ SGLD noise
// Counter index0 + i for i < n: the raw Philox words and the four normals.
__global__ __launch_bounds__(256) void k_normals(int64_t n, uint64_t index0, uint32_t tag, uint32_t step, uint64_t seed,
                                                 float* __restrict__ z, uint32_t* __restrict__ words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t idx = index0 + (uint64_t)i;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)idx, (uint32_t)(idx >> 32), tag, step), (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    if (words) reinterpret_cast<uint4*>(words)[i] = w;
    float4 o;
    box_muller_pair(w.x, w.y, o.x, o.y);
    box_muller_pair(w.z, w.w, o.z, o.w);
    reinterpret_cast<float4*>(z)[i] = o;
}

hipError_t launch_normals(int64_t n, uint64_t index0, uint32_t tag, uint32_t step, uint64_t seed, float* z,
                          uint32_t* words, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normals, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, index0, tag, step, seed, z,
                       words);
    return hipGetLastError();
}

}  // namespace cgs
