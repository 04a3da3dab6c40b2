/*
 * ORACLE (test infrastructure only).  Only tests/, the smoke check and the
 * benchmark's CPU-baseline leg may load this code; the product path never does.
 *
 * Brute-force FP64 front-to-back compositing of one view (paper Sec. 2.1,
 * Eq. 3: C(x) = sum_k alpha_k c_k prod_{i<k} (1 - alpha_i)) and its exact
 * reverse-mode derivative with respect to each Gaussian's projected
 * parameters.
 *
 * For every requested pixel the loop visits ALL Gaussians in the given depth
 * order (no tile lists, no sorting here).  A Gaussian may contribute to a
 * pixel only if the pixel's 16x16 tile lies in the Gaussian's tile rectangle
 * (decided by the FP32 skeleton), and then the renderer's truncation rules
 * apply:
 *   power = -1/2 (A dx^2 + C dy^2) - B dx dy, dx = px - u, dy = py - v,
 *           clamped to <= 0 (the conic is positive definite, so only rounding
 *           can make it positive)
 *   alpha = min(0.99, o exp(power));  alpha < 1/255 -> skipped
 *   if T (1 - alpha) < 1e-4 the walk stops before blending that Gaussian
 *   colour += alpha T c; T *= (1 - alpha); finally colour += T bg.
 * n_last is the 1-based position, among the Gaussians whose rectangle holds
 * the pixel's tile, of the last one blended (0 if none).
 *
 * A pixel is flagged ambiguous when any of its FP64 threshold tests (alpha
 * against 1/255, T(1-alpha) against 1e-4) lies within a relative margin of
 * the threshold: FP32 arithmetic may legitimately decide those differently.
 * rec_margin (optional, one per record) widens the margin of a record whose
 * FP32 alpha is known to be less accurate (an ill-conditioned footprint): its
 * alpha test uses max(margin, rec_margin[r]), and every transmittance test
 * from that record on uses the largest margin of the records blended so far,
 * since an error in an earlier alpha carries into T.
 *
 * Record layout per Gaussian (FP64): u v A B C o r g b.
 * Gradient layout matches; gradients are accumulated (+=) into grad_rec.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { int64_t rec; double alpha, T, G, og, dx, dy; int clampa, clampp; } contrib_t;

/* Arrays rec/trect are given in depth order (record j is the j-th nearest).
 * Contributor lists: when fz_rec is non-NULL and replay == 0, the records
 * blended at pixel p are written to fz_rec[fz_ptr[p] ...] (fz_ptr from the
 * out_ncontrib counts of an earlier call).  With replay != 0 the pixel
 * blends exactly the listed records in that order and takes no threshold or
 * termination decision: the frozen active set used for finite differences. */
int oc_composite(int64_t n_rec, const double* rec, const int32_t* trect,
                 int32_t W, int32_t H, const double* bg,
                 int64_t n_pix, const int32_t* pix,
                 double* out_color, double* out_T, int32_t* out_nlast, int32_t* out_amb,
                 int32_t* out_ncontrib,
                 const double* grad_color, double* grad_rec, double margin,
                 int32_t replay, const int64_t* fz_ptr, int64_t* fz_rec, const double* rec_margin)
{
    (void)W; (void)H;
    int fail = 0;
    #pragma omp parallel
    {
        int64_t cap = 1024;
        contrib_t* list = (contrib_t*)malloc(sizeof(contrib_t) * (size_t)cap);
        if (!list) {
            #pragma omp atomic write
            fail = 1;
        }
        #pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < n_pix; ++p) {
            if (!list) continue;
            const int px = pix[2 * p], py = pix[2 * p + 1];
            const int tx = px >> 4, ty = py >> 4;
            double T = 1.0, col[3] = {0.0, 0.0, 0.0};
            int64_t pos = 0, nlast = 0, nc = 0, nblend = 0;
            int amb = 0;
            double tmargin = margin;   /* margin of the transmittance test */
            const int64_t jend = replay ? fz_ptr[p + 1] - fz_ptr[p] : n_rec;
            for (int64_t j = 0; j < jend; ++j) {
                const int64_t r = replay ? fz_rec[fz_ptr[p] + j] : j;
                const int32_t* tr = trect + 4 * r;
                if (!replay && (tx < tr[0] || tx >= tr[2] || ty < tr[1] || ty >= tr[3])) continue;
                ++pos;
                const double* g = rec + 9 * r;
                const double dx = (double)px - g[0], dy = (double)py - g[1];
                double power = -0.5 * (g[2] * dx * dx + g[4] * dy * dy) - g[3] * dx * dy;
                int clampp = 0;
                if (power > 0.0) { power = 0.0; clampp = 1; }
                const double G = exp(power);
                const double og = g[5] * G;
                int clampa = 0;
                double alpha = og;
                if (alpha > 0.99) { alpha = 0.99; clampa = 1; }
                const double amargin = (rec_margin && rec_margin[r] > margin) ? rec_margin[r] : margin;
                if (fabs(alpha - 1.0 / 255.0) <= amargin * (1.0 / 255.0)) amb = 1;
                if (!replay && alpha < 1.0 / 255.0) continue;
                if (amargin > tmargin) tmargin = amargin;
                const double Tn = T * (1.0 - alpha);
                if (fabs(Tn - 1e-4) <= tmargin * 1e-4) amb = 1;
                if (!replay && Tn < 1e-4) break;
                if (fz_rec && !replay) fz_rec[fz_ptr[p] + nblend] = r;
                ++nblend;
                for (int c = 0; c < 3; ++c) col[c] += alpha * T * g[6 + c];
                if (grad_color) {
                    if (nc == cap) {
                        cap *= 2;
                        contrib_t* nl = (contrib_t*)realloc(list, sizeof(contrib_t) * (size_t)cap);
                        if (!nl) {
                            #pragma omp atomic write
                            fail = 1;
                            break;
                        }
                        list = nl;
                    }
                    contrib_t* e = &list[nc++];
                    e->rec = r; e->alpha = alpha; e->T = T; e->G = G; e->og = og;
                    e->dx = dx; e->dy = dy; e->clampa = clampa; e->clampp = clampp;
                }
                T = Tn;
                nlast = pos;
            }
            for (int c = 0; c < 3; ++c) out_color[3 * p + c] = col[c] + T * bg[c];
            out_T[p] = T;
            out_nlast[p] = (int32_t)nlast;
            out_amb[p] = amb;
            if (out_ncontrib) out_ncontrib[p] = (int32_t)nblend;
            if (grad_color) {
                /* Reverse sweep with stored T_k.  behind = colour composited
                 * behind Gaussian k, normalised to unit transmittance at k+1:
                 * behind_{k-1} = alpha_k c_k + (1 - alpha_k) behind_k, starting
                 * from the background.  dC/dalpha_k = T_k (c_k - behind_k),
                 * dC/dc_k = alpha_k T_k. */
                const double* gc = grad_color + 3 * p;
                double behind[3] = {bg[0], bg[1], bg[2]};
                for (int64_t k = nc - 1; k >= 0; --k) {
                    const contrib_t* e = &list[k];
                    const double* g = rec + 9 * e->rec;
                    double* gr = grad_rec + 9 * e->rec;
                    double dalpha = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        double dcol = e->alpha * e->T * gc[c];
                        #pragma omp atomic
                        gr[6 + c] += dcol;
                        dalpha += gc[c] * e->T * (g[6 + c] - behind[c]);
                        behind[c] = e->alpha * g[6 + c] + (1.0 - e->alpha) * behind[c];
                    }
                    if (e->clampa) continue;           /* min(0.99, .) saturated */
                    double dop = dalpha * e->G;       /* d alpha / d o = G */
                    #pragma omp atomic
                    gr[5] += dop;
                    if (e->clampp) continue;           /* power clamped at 0 */
                    double dpow = dalpha * e->og;     /* d alpha / d power = o G */
                    double du = dpow * (g[2] * e->dx + g[3] * e->dy);
                    double dv = dpow * (g[4] * e->dy + g[3] * e->dx);
                    double dA = dpow * (-0.5 * e->dx * e->dx);
                    double dB = dpow * (-e->dx * e->dy);
                    double dC = dpow * (-0.5 * e->dy * e->dy);
                    #pragma omp atomic
                    gr[0] += du;
                    #pragma omp atomic
                    gr[1] += dv;
                    #pragma omp atomic
                    gr[2] += dA;
                    #pragma omp atomic
                    gr[3] += dB;
                    #pragma omp atomic
                    gr[4] += dC;
                }
            }
        }
        free(list);
    }
    return fail ? -1 : 0;
}
