/*
 * ORACLE (test infrastructure only).  Only tests/, the smoke check and the
 * benchmark's CPU-baseline leg may load this code; the product path never does.
 *
 * The FP32 "discrete skeleton" of the tile renderer: for each Gaussian seen
 * from one camera, the cull decision, the depth sort key and the tile
 * rectangle.  These are integer outcomes decided by floating point, so the
 * oracle takes them in FP32 with exactly the operation sequence fixed below
 * (every operation one IEEE round-to-nearest step, no contraction, exp by
 * an own Cody-Waite + Taylor routine).  The HIP path implements the same
 * sequence independently; the two must agree bit for bit.  The continuous
 * values the oracle composites with are recomputed in FP64 elsewhere.
 *
 * What is decided (paper Sec. 2.1, Eq. 1-3; the tile binning is that of the
 * 3DGS renderer the paper builds on):
 *   camera point  x_c = R mu + t                (row sums left to right)
 *   cull          !(z_c > 0.2)
 *   depth key     IEEE bits of z_c
 *   scale         s = exp(ls)                    (ks_exp below)
 *   rotation      R(q/|q|), Eq. 2
 *   Sigma3D       M M^T, M = R(q) diag(s)        (Eq. 2)
 *   Jacobian      J of the pinhole projection, x/z and y/z clamped to
 *                 +-1.3 * (W/2)/fx and +-1.3 * (H/2)/fy
 *   Sigma2D diag  a = (T Sigma3D T^T)_00 + 0.3, c = (...)_11 + 0.3, T = J W
 *   mean2D        u = fx*(x/z)+cx, v = fy*(y/z)+cy
 *   pixel rect    [ceil(u-3 sqrt a), floor(u+3 sqrt a)] clipped to the image,
 *                 same in y; empty -> culled
 *   tile rect     [x_lo>>4, (x_hi>>4)+1) x [y_lo>>4, (y_hi>>4)+1)
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* exp(x) for the skeleton: x = n ln2 + r with ln2 split in a 16-bit head and
 * a tail (Cody & Waite's additive range reduction), |r| <= ln2/2, exp(r) by
 * the degree-7 Taylor polynomial in Horner form with fused multiply-adds,
 * result scaled by 2^n.  Input clamped to [-80,80] so every result is a
 * normal float.  Coefficients are 1/k! rounded to float. */
static float ks_exp(float x)
{
    const float LOG2E = 1.44269502162933349609375f;      /* float(1/ln 2) */
    const float LN2_HI = 0.693145751953125f;              /* ln2 to 16 bits */
    const float LN2_LO = 1.428606765330187045037746429443359375e-06f; /* float(ln2 - LN2_HI) */
    if (x > 80.0f) x = 80.0f;
    if (x < -80.0f) x = -80.0f;
    float n = rintf(x * LOG2E);
    float r = x - n * LN2_HI;
    r = r - n * LN2_LO;
    float p = 1.98412701138295233249664306640625e-04f;    /* 1/5040 */
    p = fmaf(p, r, 1.3888889225199818611145019531250e-03f); /* 1/720 */
    p = fmaf(p, r, 8.3333337679505348205566406250000e-03f); /* 1/120 */
    p = fmaf(p, r, 4.1666667908430099487304687500000e-02f); /* 1/24 */
    p = fmaf(p, r, 1.6666667163372039794921875000000e-01f); /* 1/6 */
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)n);
}

float ok_exp(float x) { return ks_exp(x); }

/* One Gaussian.  cam: fx fy cx cy R00..R22,t (row-major 3x4), W, H.
 * row: ls0 ls1 ls2 qw qx qy qz.  Writes key and tile rect; returns 1 if kept. */
static int ks_one(const float* mu, const float* row, const float* cam, int W, int H,
                  uint32_t* key, uint16_t* trect)
{
    const float fx = cam[0], fy = cam[1], cx = cam[2], cy = cam[3];
    const float* Rt = cam + 4;
    float xc = Rt[0] * mu[0]; xc = xc + Rt[1] * mu[1]; xc = xc + Rt[2] * mu[2]; xc = xc + Rt[3];
    float yc = Rt[4] * mu[0]; yc = yc + Rt[5] * mu[1]; yc = yc + Rt[6] * mu[2]; yc = yc + Rt[7];
    float zc = Rt[8] * mu[0]; zc = zc + Rt[9] * mu[1]; zc = zc + Rt[10] * mu[2]; zc = zc + Rt[11];
    trect[0] = trect[1] = trect[2] = trect[3] = 0;
    *key = 0xFFFFFFFFu;
    if (!(zc > 0.2f)) return 0;
    uint32_t zb; memcpy(&zb, &zc, 4);

    float s0 = ks_exp(row[0]), s1 = ks_exp(row[1]), s2 = ks_exp(row[2]);
    float qw = row[3], qx = row[4], qy = row[5], qz = row[6];
    float n2 = qw * qw; n2 = n2 + qx * qx; n2 = n2 + qy * qy; n2 = n2 + qz * qz;
    if (n2 > 0.0f) {
        float nn = sqrtf(n2);
        qw = qw / nn; qx = qx / nn; qy = qy / nn; qz = qz / nn;
    } else {
        qw = 1.0f; qx = qy = qz = 0.0f;
    }
    /* Rotation matrix of the unit quaternion (w,x,y,z). */
    float r00 = 1.0f - 2.0f * (qy * qy + qz * qz);
    float r01 = 2.0f * (qx * qy - qw * qz);
    float r02 = 2.0f * (qx * qz + qw * qy);
    float r10 = 2.0f * (qx * qy + qw * qz);
    float r11 = 1.0f - 2.0f * (qx * qx + qz * qz);
    float r12 = 2.0f * (qy * qz - qw * qx);
    float r20 = 2.0f * (qx * qz - qw * qy);
    float r21 = 2.0f * (qy * qz + qw * qx);
    float r22 = 1.0f - 2.0f * (qx * qx + qy * qy);
    float M[3][3] = {{r00 * s0, r01 * s1, r02 * s2},
                     {r10 * s0, r11 * s1, r12 * s2},
                     {r20 * s0, r21 * s1, r22 * s2}};
    float S[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            float acc = M[i][0] * M[j][0];
            acc = acc + M[i][1] * M[j][1];
            acc = acc + M[i][2] * M[j][2];
            S[i][j] = acc;
        }
    float tx = xc / zc, ty = yc / zc;
    float limx = 1.3f * ((0.5f * (float)W) / fx);
    float limy = 1.3f * ((0.5f * (float)H) / fy);
    float txc = fminf(limx, fmaxf(-limx, tx));
    float tyc = fminf(limy, fmaxf(-limy, ty));
    float j00 = fx / zc, j02 = -(fx * txc) / zc;
    float j11 = fy / zc, j12 = -(fy * tyc) / zc;
    float T[2][3];
    for (int j = 0; j < 3; ++j) {
        T[0][j] = j00 * Rt[0 + j] + j02 * Rt[8 + j];
        T[1][j] = j11 * Rt[4 + j] + j12 * Rt[8 + j];
    }
    float d2[2];
    for (int a = 0; a < 2; ++a) {
        float U[3];
        for (int j = 0; j < 3; ++j) {
            float acc = T[a][0] * S[0][j];
            acc = acc + T[a][1] * S[1][j];
            acc = acc + T[a][2] * S[2][j];
            U[j] = acc;
        }
        float acc = U[0] * T[a][0];
        acc = acc + U[1] * T[a][1];
        acc = acc + U[2] * T[a][2];
        d2[a] = acc + 0.3f;
    }
    float u = fx * tx + cx;
    float v = fy * ty + cy;
    float ex = 3.0f * sqrtf(d2[0]);
    float ey = 3.0f * sqrtf(d2[1]);
    float xlo = fmaxf(ceilf(u - ex), 0.0f);
    float xhi = fminf(floorf(u + ex), (float)(W - 1));
    float ylo = fmaxf(ceilf(v - ey), 0.0f);
    float yhi = fminf(floorf(v + ey), (float)(H - 1));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return 0;
    int ixlo = (int)xlo, ixhi = (int)xhi, iylo = (int)ylo, iyhi = (int)yhi;
    trect[0] = (uint16_t)(ixlo >> 4);
    trect[1] = (uint16_t)(iylo >> 4);
    trect[2] = (uint16_t)((ixhi >> 4) + 1);
    trect[3] = (uint16_t)((iyhi >> 4) + 1);
    *key = zb;
    return 1;
}

/* rows: [n][7] float (ls3, q4) already gathered per Gaussian. */
void ok_keyspec(int64_t n, const float* means, const float* rows, const float* cam,
                int32_t W, int32_t H, uint32_t* key, uint16_t* trect, uint8_t* kept)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        kept[i] = (uint8_t)ks_one(means + 3 * i, rows + 7 * i, cam, W, H, key + i, trect + 4 * i);
}
