// Per-Gaussian math shared by the forward and backward kernels of libcgs.
//
// Two kinds of arithmetic live here:
//  * the FP32 "skeleton" (skel_* and the marked blocks of gaussian_shape /
//    project_view): it decides integers -- culling, depth keys, tile
//    rectangles -- so its operation sequence is fixed (one IEEE rounding per
//    written operation, no contraction, exp by Cody-Waite reduction and a
//    Taylor polynomial) and reproducible bit for bit by any IEEE FP32
//    implementation of the same sequence;
//  * continuous FP32 math (conic, colour, compositing), free to use fused
//    multiply-adds and the hardware exp, with an FP64 island for the 2x2
//    determinant and inverse of near-degenerate projected covariances.
#pragma once

#include "cgs_internal.h"

namespace cgs {

constexpr float kMinAlpha = 1.0f / 255.0f;   // alpha below this is skipped
constexpr float kMaxAlpha = 0.99f;           // alpha saturates here
constexpr float kMinT = 1e-4f;               // stop before T would drop below this
constexpr float kNear = 0.2f;                // near-plane cull
constexpr float kBlur = 0.3f;                // low-pass added to Sigma2D

// Real orthonormal spherical harmonics with the Condon-Shortley phase, as
// polynomials in the unit direction (x, y, z); index j = l*l + l + m.
// Normalisation constants in closed form:
constexpr float kY00 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kY1 = 0.4886025119029199f;     // sqrt(3/(4 pi))
constexpr float kY2a = 1.0925484305920792f;    // sqrt(15/(4 pi))
constexpr float kY2b = 0.31539156525252005f;   // sqrt(5/(16 pi))
constexpr float kY2c = 0.5462742152960396f;    // sqrt(15/(16 pi))
constexpr float kY3a = 0.5900435899266435f;    // sqrt(35/(32 pi))
constexpr float kY3b = 2.890611442640554f;     // sqrt(105/(4 pi))
constexpr float kY3c = 0.4570457994644658f;    // sqrt(21/(32 pi))
constexpr float kY3d = 0.3731763325901154f;    // sqrt(7/(16 pi))
constexpr float kY3e = 1.445305721320277f;     // sqrt(105/(16 pi))

// ------------------------------------------------------------ skeleton exp
// exp(x) = 2^n p(r): n = rint(x / ln 2), r = x - n ln2 with ln 2 split in a
// 16-bit head and a tail (Cody & Waite), p the degree-7 Taylor polynomial of
// exp (coefficients 1/k! rounded to float) in Horner form with fused
// multiply-adds.  x is clamped to [-80, 80] so results stay normal.
__device__ inline float skel_exp(float x) {
#pragma clang fp contract(off)
    x = x > 80.0f ? 80.0f : x;
    x = x < -80.0f ? -80.0f : x;
    const float n = __builtin_rintf(x * 1.44269502162933349609375f);
    float r = x - n * 0.693145751953125f;
    r = r - n * 1.428606765330187045037746429443359375e-06f;
    float p = 1.98412701138295233249664306640625e-04f;
    p = __builtin_fmaf(p, r, 1.388888922519981861114501953125e-03f);
    p = __builtin_fmaf(p, r, 8.333333767950534820556640625e-03f);
    p = __builtin_fmaf(p, r, 4.16666679084300994873046875e-02f);
    p = __builtin_fmaf(p, r, 1.6666667163372039794921875e-01f);
    p = __builtin_fmaf(p, r, 0.5f);
    p = __builtin_fmaf(p, r, 1.0f);
    p = __builtin_fmaf(p, r, 1.0f);
    return __builtin_ldexpf(p, (int)n);
}

// ---------------------------------------------------------- Gaussian state
struct GaussParams {
    float mean[3];
    float ls[3];
    float q[4];     // (w, x, y, z) as stored
    float logit;
    float sh[48];   // [coef][rgb]
};

// N consecutive codebook values starting at element `off` of `base`, read
// with 16-byte loads (caller guarantees alignment and N * size % 16 == 0).
template <int DT, int N>
__device__ inline void load_vec(const void* base, int64_t off, float* out) {
    if constexpr (DT == CGS_BF16) {
        static_assert(N % 8 == 0, "BF16 vector rows come in 8s");
        const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + off);
#pragma unroll
        for (int i = 0; i < N / 8; ++i) {
            const uint4 q = p[i];
            const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                out[8 * i + 2 * k] = __uint_as_float(wv[k] << 16);
                out[8 * i + 2 * k + 1] = __uint_as_float(wv[k] & 0xffff0000u);
            }
        }
    } else {
        static_assert(N % 4 == 0, "FP32 vector rows come in 4s");
        const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + off);
#pragma unroll
        for (int i = 0; i < N / 4; ++i) {
            const float4 q = p[i];
            out[4 * i] = q.x; out[4 * i + 1] = q.y; out[4 * i + 2] = q.z; out[4 * i + 3] = q.w;
        }
    }
}

// Returns false (and loads nothing) when an index is outside its codebook:
// such a Gaussian is treated as culled and receives zero gradient.
template <int DT, int SHD>
__device__ inline bool load_gaussian(const SceneDesc& sd, int64_t g, GaussParams& gp, bool vec) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    const int64_t ksr = sd.idx_sr[g];
    const int64_t ksh = sd.idx_sh[g];
    if (ksr < 0 || ksr >= sd.sr_rows || ksh < 0 || ksh >= sd.sh_rows) return false;
    gp.mean[0] = sd.means[3 * g + 0];
    gp.mean[1] = sd.means[3 * g + 1];
    gp.mean[2] = sd.means[3 * g + 2];
    const int64_t bsr = ksr * sd.sr_stride + sd.sr_col0;
    const int64_t bsh = ksh * sd.sh_stride + sd.sh_col0;
    if constexpr (SHD == 3) {
        if (vec) {      // host-checked: aligned rows, opacity in the SR row
            float sr[8];
            load_vec<DT, 8>(sd.sr, bsr, sr);
            gp.ls[0] = sr[0]; gp.ls[1] = sr[1]; gp.ls[2] = sr[2];
            gp.q[0] = sr[3]; gp.q[1] = sr[4]; gp.q[2] = sr[5]; gp.q[3] = sr[6];
            gp.logit = sr[7];
            load_vec<DT, 48>(sd.sh, bsh, gp.sh);
            return true;
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) gp.ls[i] = load_cb<DT>(sd.sr, bsr + i);
#pragma unroll
    for (int i = 0; i < 4; ++i) gp.q[i] = load_cb<DT>(sd.sr, bsr + 3 + i);
    gp.logit = sd.opacity_mode ? load_cb<DT>(sd.sr, bsr + 7) : sd.opacity[g];
#pragma unroll
    for (int i = 0; i < 3 * NCO; ++i) gp.sh[i] = load_cb<DT>(sd.sh, bsh + i);
    return true;
}

// The same for a Gaussian whose codebook row is already known (single
// codebook, row in range): the row loads do not wait for the index load;
// the Gaussian is valid iff its index equals that row.
template <int DT, int SHD>
__device__ inline bool load_gaussian_row(const SceneDesc& sd, int64_t g, int64_t row, GaussParams& gp, bool vec) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    const bool ok = sd.idx_sr[g] == row && sd.idx_sh[g] == row;
    gp.mean[0] = sd.means[3 * g + 0];
    gp.mean[1] = sd.means[3 * g + 1];
    gp.mean[2] = sd.means[3 * g + 2];
    const int64_t bsr = row * sd.sr_stride + sd.sr_col0;
    const int64_t bsh = row * sd.sh_stride + sd.sh_col0;
    if constexpr (SHD == 3) {
        if (vec) {
            float sr[8];
            load_vec<DT, 8>(sd.sr, bsr, sr);
            gp.ls[0] = sr[0]; gp.ls[1] = sr[1]; gp.ls[2] = sr[2];
            gp.q[0] = sr[3]; gp.q[1] = sr[4]; gp.q[2] = sr[5]; gp.q[3] = sr[6];
            gp.logit = sr[7];
            load_vec<DT, 48>(sd.sh, bsh, gp.sh);
            return ok;
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) gp.ls[i] = load_cb<DT>(sd.sr, bsr + i);
#pragma unroll
    for (int i = 0; i < 4; ++i) gp.q[i] = load_cb<DT>(sd.sr, bsr + 3 + i);
    gp.logit = sd.opacity_mode ? load_cb<DT>(sd.sr, bsr + 7) : sd.opacity[g];
#pragma unroll
    for (int i = 0; i < 3 * NCO; ++i) gp.sh[i] = load_cb<DT>(sd.sh, bsh + i);
    return ok;
}

// View-independent shape: scale, unit quaternion, R(q), M = R S, Sigma = M M^T.
struct GaussShape {
    float s[3];
    float qn[4];
    float qlen;
    float R[3][3];
    float M[3][3];
    float S[3][3];
};

__device__ inline void gaussian_shape(const GaussParams& gp, GaussShape& o) {
#pragma clang fp contract(off)
    o.s[0] = skel_exp(gp.ls[0]);
    o.s[1] = skel_exp(gp.ls[1]);
    o.s[2] = skel_exp(gp.ls[2]);
    float w = gp.q[0], x = gp.q[1], y = gp.q[2], z = gp.q[3];
    float n2 = w * w;
    n2 = n2 + x * x;
    n2 = n2 + y * y;
    n2 = n2 + z * z;
    if (n2 > 0.0f) {
        const float len = __builtin_sqrtf(n2);
        o.qlen = len;
        w = w / len; x = x / len; y = y / len; z = z / len;
    } else {
        o.qlen = 0.0f;
        w = 1.0f; x = 0.0f; y = 0.0f; z = 0.0f;
    }
    o.qn[0] = w; o.qn[1] = x; o.qn[2] = y; o.qn[3] = z;
    o.R[0][0] = 1.0f - 2.0f * (y * y + z * z);
    o.R[0][1] = 2.0f * (x * y - w * z);
    o.R[0][2] = 2.0f * (x * z + w * y);
    o.R[1][0] = 2.0f * (x * y + w * z);
    o.R[1][1] = 1.0f - 2.0f * (x * x + z * z);
    o.R[1][2] = 2.0f * (y * z - w * x);
    o.R[2][0] = 2.0f * (x * z - w * y);
    o.R[2][1] = 2.0f * (y * z + w * x);
    o.R[2][2] = 1.0f - 2.0f * (x * x + y * y);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) o.M[i][j] = o.R[i][j] * o.s[j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            float acc = o.M[i][0] * o.M[j][0];
            acc = acc + o.M[i][1] * o.M[j][1];
            acc = acc + o.M[i][2] * o.M[j][2];
            o.S[i][j] = acc;
            o.S[j][i] = acc;
        }
}

// ------------------------------------------------------------- projection
struct ViewProj {
    float xc, yc, zc;
    float tx, ty;          // x/z, y/z
    float txc, tyc;        // clamped
    bool clx, cly;         // clamp active
    float j00, j02, j11, j12;
    float T[2][3];         // J W
    float U0[3];           // (T Sigma) row 0
    float a, b, c;         // Sigma2D (+ 0.3 on the diagonal)
    float u, v;
    int tx0, ty0, tx1, ty1;
};

// Camera point, cull, Jacobian, Sigma2D and the tile rectangle.  Returns false
// when the Gaussian is culled (behind the near plane or off the image).
// The camera point W mu + t, in the skeleton's order of operations.
__device__ inline void camera_point(const ViewDesc& vd, const float* mu, float& xc, float& yc, float& zc) {
#pragma clang fp contract(off)
    const float* Rt = vd.Rt;
    xc = Rt[0] * mu[0]; xc = xc + Rt[1] * mu[1]; xc = xc + Rt[2] * mu[2]; xc = xc + Rt[3];
    yc = Rt[4] * mu[0]; yc = yc + Rt[5] * mu[1]; yc = yc + Rt[6] * mu[2]; yc = yc + Rt[7];
    zc = Rt[8] * mu[0]; zc = zc + Rt[9] * mu[1]; zc = zc + Rt[10] * mu[2]; zc = zc + Rt[11];
}

__device__ inline bool project_view(const ViewDesc& vd, const float* mu, const GaussShape& sh, ViewProj& p) {
#pragma clang fp contract(off)
    const float* Rt = vd.Rt;
    float xc, yc, zc;
    camera_point(vd, mu, xc, yc, zc);
    p.xc = xc; p.yc = yc; p.zc = zc;
    if (!(zc > kNear)) return false;
    const float tx = xc / zc, ty = yc / zc;
    const float limx = vd.limx, limy = vd.limy;
    const float txc = fminf(limx, fmaxf(-limx, tx));
    const float tyc = fminf(limy, fmaxf(-limy, ty));
    p.tx = tx; p.ty = ty; p.txc = txc; p.tyc = tyc;
    p.clx = !(tx >= -limx && tx <= limx);
    p.cly = !(ty >= -limy && ty <= limy);
    p.j00 = vd.fx / zc;
    p.j02 = -(vd.fx * txc) / zc;
    p.j11 = vd.fy / zc;
    p.j12 = -(vd.fy * tyc) / zc;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        p.T[0][j] = p.j00 * Rt[0 + j] + p.j02 * Rt[8 + j];
        p.T[1][j] = p.j11 * Rt[4 + j] + p.j12 * Rt[8 + j];
    }
    float d2[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        float U[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float acc = p.T[a][0] * sh.S[0][j];
            acc = acc + p.T[a][1] * sh.S[1][j];
            acc = acc + p.T[a][2] * sh.S[2][j];
            U[j] = acc;
        }
        if (a == 0) { p.U0[0] = U[0]; p.U0[1] = U[1]; p.U0[2] = U[2]; }
        float acc = U[0] * p.T[a][0];
        acc = acc + U[1] * p.T[a][1];
        acc = acc + U[2] * p.T[a][2];
        d2[a] = acc + kBlur;
    }
    p.a = d2[0];
    p.c = d2[1];
    {
        float acc = p.U0[0] * p.T[1][0];
        acc = acc + p.U0[1] * p.T[1][1];
        acc = acc + p.U0[2] * p.T[1][2];
        p.b = acc;
    }
    p.u = vd.fx * tx + vd.cx;
    p.v = vd.fy * ty + vd.cy;
    const float ex = 3.0f * __builtin_sqrtf(p.a);
    const float ey = 3.0f * __builtin_sqrtf(p.c);
    const float xlo = fmaxf(__builtin_ceilf(p.u - ex), 0.0f);
    const float xhi = fminf(__builtin_floorf(p.u + ex), (float)(vd.W - 1));
    const float ylo = fmaxf(__builtin_ceilf(p.v - ey), 0.0f);
    const float yhi = fminf(__builtin_floorf(p.v + ey), (float)(vd.H - 1));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return false;
    p.tx0 = ((int)xlo) >> 4;
    p.ty0 = ((int)ylo) >> 4;
    p.tx1 = (((int)xhi) >> 4) + 1;
    p.ty1 = (((int)yhi) >> 4) + 1;
    return true;
}

// Conic = inverse of [[a, b], [b, c]].  The FP32 determinant loses the
// leading digits when the footprint is very elongated (a c ~ b^2); then
// determinant and inverse are taken in FP64.  Returns true in that case (a
// near-degenerate footprint).
__device__ inline bool conic_of(float a, float b, float c, float& A, float& B, float& C) {
    const float det = a * c - b * b;
    if (det > 0x1p-10f * (a * c)) {
        const float id = 1.0f / det;
        A = c * id; B = -b * id; C = a * id;
        return false;
    }
    const double da = a, db = b, dc = c;
    const double dd = da * dc - db * db;
    const double id = 1.0 / dd;
    A = (float)(dc * id); B = (float)(-db * id); C = (float)(da * id);
    return true;
}

// The FP64 inverse itself (for the FP64 chain rule of near-degenerate
// footprints).
__device__ inline void conic_of_f64(float a, float b, float c, double& A, double& B, double& C) {
    const double da = a, db = b, dc = c;
    const double id = 1.0 / (da * dc - db * db);
    A = dc * id; B = -db * id; C = da * id;
}

// ---------------------------------------------------------------- colour
template <int SHD>
__device__ inline void sh_basis(float x, float y, float z, float* Y) {
    Y[0] = kY00;
    if constexpr (SHD >= 1) {
        Y[1] = -kY1 * y;
        Y[2] = kY1 * z;
        Y[3] = -kY1 * x;
    }
    if constexpr (SHD >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kY2a * (x * y);
        Y[5] = -kY2a * (y * z);
        Y[6] = kY2b * (2.0f * zz - xx - yy);
        Y[7] = -kY2a * (x * z);
        Y[8] = kY2c * (xx - yy);
        if constexpr (SHD >= 3) {
            Y[9] = -kY3a * y * (3.0f * xx - yy);
            Y[10] = kY3b * (x * y * z);
            Y[11] = -kY3c * y * (4.0f * zz - xx - yy);
            Y[12] = kY3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -kY3c * x * (4.0f * zz - xx - yy);
            Y[14] = kY3e * z * (xx - yy);
            Y[15] = -kY3a * x * (xx - 3.0f * yy);
        }
    }
}

// colour = max(0, sum_j Y_j(dir) k_j + 1/2), dir = (mean - campos)/|.|.
// pre (optional) receives the unclamped values.
template <int SHD>
__device__ inline void sh_colour(const ViewDesc& vd, const GaussParams& gp, float* col, float* pre) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    float dx = gp.mean[0] - vd.campos[0], dy = gp.mean[1] - vd.campos[1], dz = gp.mean[2] - vd.campos[2];
    const float il = rsqrtf(dx * dx + dy * dy + dz * dz);
    dx *= il; dy *= il; dz *= il;
    float Y[16];
    sh_basis<SHD>(dx, dy, dz, Y);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.5f;
#pragma unroll
        for (int j = 0; j < NCO; ++j) acc = fmaf(Y[j], gp.sh[3 * j + ch], acc);
        if (pre) pre[ch] = acc;
        col[ch] = fmaxf(acc, 0.0f);
    }
}

// ------------------------------------------------------------- compositing
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// alpha of one (pixel, Gaussian) pair.  Records hold the conic pre-scaled by
// log2(e): g = (u, v, -A/2 log2e, -B log2e), c = (-C/2 log2e, opacity, r, g),
// so power log2e = (g.z dx + g.w dy) dx + c.x dy^2 and exp(power) is one
// hardware exp2.  power is clamped to <= 0 (rounding residue of a positive-
// definite form); alpha = min(0.99, o exp(power)).  Forward and backward call
// this same function so both take identical decisions.
__device__ inline float blend_alpha(float dx, float dy, const float4& g, const float4& c, float& G, bool& pclamp) {
#pragma clang fp contract(off)
    const float t = __builtin_fmaf(g.z, dx, g.w * dy);
    float pw = __builtin_fmaf(t, dx, (c.x * dy) * dy);
    pclamp = pw > 0.0f;
    pw = fminf(pw, 0.0f);
    G = __builtin_amdgcn_exp2f(pw);
    const float og = c.y * G;
    return og < kMaxAlpha ? og : kMaxAlpha;
}

// Minimum over the rectangle [x0,x1] x [y0,y1] of the positive-definite
// quadratic form f(p) = (p-m)^T K (p-m), K = [[A, B], [B, C]]: zero if m is
// inside, otherwise the least of the four edge minima (on an edge the form is
// a 1-D quadratic, minimised at its clamped vertex).
__device__ inline float rect_min_form(float A, float B, float C, float mx, float my, float x0, float x1, float y0,
                                      float y1) {
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.f;
    const float iA = 1.f / A, iC = 1.f / C;
    float best = 3.0e38f;
    const float xs[2] = {x0, x1}, ys[2] = {y0, y1};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dx = xs[e] - mx;
        const float dy = fminf(fmaxf(-B * dx * iC, y0 - my), y1 - my);
        best = fminf(best, A * dx * dx + 2.f * B * dx * dy + C * dy * dy);
        const float ey = ys[e] - my;
        const float ex = fminf(fmaxf(-B * ey * iA, x0 - mx), x1 - mx);
        best = fminf(best, A * ex * ex + 2.f * B * ex * ey + C * ey * ey);
    }
    return best;
}

// Which 8x8 quadrants of a 16x16 tile (pixel origin x0, y0; last valid pixel
// xm, ym) can the record reach with alpha >= 1/255?  Bit k = quadrant
// (k & 1, k >> 1).  Exact alpha (on the stored record values) at a pixel p is
// o exp(-f(p)/2) with f the conic form; it reaches lo = (1/255)(1 - 1e-3)
// only where f <= rho = 2 ln(o/lo).  A quadrant whose pixel rectangle has
// min f > rho (with a 1e-4 relative safety margin for this FP32 evaluation)
// holds no pixel with exact alpha >= lo, so the FP32 alpha of blend_alpha
// (relative error ~1e-6) stays below 1/255 there and every pair would be
// skipped anyway: skipping such quadrants changes no result.
__device__ inline uint32_t quadrant_mask(const float4& g, const float4& c, float x0, float y0, float xm, float ym) {
    const float lo = kMinAlpha * 0.999f;
    const float o = c.y;
    if (!(o > lo)) return 0u;
    const float A = -2.f * kLn2 * g.z, B = -kLn2 * g.w, C = -2.f * kLn2 * c.x;
    if (!(A > 0.f && C > 0.f && A * C - B * B > 0.f)) return 0xfu;     // no claim: keep all
    const float rho = 2.f * __logf(o / lo) * 1.0001f + 1e-4f;
    uint32_t m = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float qx0 = x0 + 8.f * (float)(k & 1), qy0 = y0 + 8.f * (float)(k >> 1);
        if (qx0 > xm || qy0 > ym) continue;
        const float qx1 = fminf(qx0 + 7.f, xm), qy1 = fminf(qy0 + 7.f, ym);
        if (rect_min_form(A, B, C, g.x, g.y, qx0, qx1, qy0, qy1) <= rho) m |= 1u << k;
    }
    return m;
}

// The tile a wavefront shades.  Order 0: row-major.  Order 1 groups
// consecutive tiles on one XCD: the dispatcher deals workgroups to the 8 XCDs
// round-robin, so workgroup b runs on XCD b % 8; XCD x gets a contiguous range
// of tile groups so neighbouring tiles (which share Gaussians) hit the same
// L2.  Order 2: heaviest tiles first (tiles sorted by descending list length),
// so the longest lists start early and do not form the tail of the launch.
__device__ inline int64_t tile_index(const BatchDesc* d, int64_t b, int64_t nb, int w, int wpb) {
    if (d->tile_order == 2) {
        const int64_t i = b * wpb + w;
        return i < d->n_tiles ? (int64_t)d->tile_perm[i] : d->n_tiles;
    }
    if (d->tile_order == 1) {
        const int64_t q = nb / 8, rm = nb % 8;
        const int64_t x = b % 8, k = b / 8;
        b = x * q + (x < rm ? x : rm) + k;
    }
    return b * wpb + w;
}

// Persistent blends: a resident grid whose wavefronts take tiles from
// queues (atomic counters) until they run dry.  A workgroup uses the queue of
// its XCD (blockIdx mod 8, the dispatch order), which hands out every 8th
// position of the tile order; the position maps to a tile through the
// heavy-first permutation (tile order 2) or directly.  fetch_pos issues the
// atomic (lane 0) and returns without waiting; tile_at reads the result.
__device__ inline uint32_t fetch_pos(unsigned long long* q, int lane) {
    uint32_t t = 0xffffffffu;
    if (lane == 0) t = (uint32_t)atomicAdd(&q[(blockIdx.x % kQueues) * kQueueStride], 1ull);
    return t;
}

__device__ inline int64_t tile_at(const BatchDesc* d, uint32_t fetched) {
    const uint64_t pos = (uint64_t)__builtin_amdgcn_readfirstlane(fetched) * kQueues + blockIdx.x % kQueues;
    if (pos >= (uint64_t)d->n_tiles) return d->n_tiles;
    return d->tile_order == 2 ? (int64_t)d->tile_perm[pos] : (int64_t)pos;
}

// A wavefront that found its queue dry retires; the last of the launch's
// `waves` wavefronts resets the queues for the next launch.
__device__ inline void retire_wave(unsigned long long* q, unsigned long long* done, unsigned long long waves,
                                   int lane) {
    if (lane == 0) {
        const unsigned long long d = atomicAdd(done, 1ull);
        if (d + 1ull == waves) {
            for (int x = 0; x < kQueues; ++x) atomicExch(&q[x * kQueueStride], 0ull);
            atomicExch(done, 0ull);
        }
    }
}

}  // namespace cgs
