/*
 * cgs.h -- C-ABI of libcgs, the MI355X (gfx950) hot path of codebook-indexed,
 * differentiable tile-based 3D Gaussian splatting.
 *
 * Problem statement (paper Sec. 4.1-4.4): the state is S = {G, C}; every
 * Gaussian g_i holds a mean p_i and integer indices into the codebooks C
 * (SR: scale + quaternion rows, SH: spherical-harmonic colour rows; Sec. 4.1,
 * Fig. 4).  One training step renders I_P(G, C) for a camera pose P (Sec. 4.2,
 * posterior) and needs the gradient of the loss with respect to every
 * differentiable parameter S_diff -- all parameters except the indices
 * (Sec. 4.4, parameter update).  The render is Eq. 1-3 of Sec. 2.1.
 *
 * Conventions for every call:
 *  - Pointers documented "device" are HIP device memory owned by the caller;
 *    the library never allocates, frees or retains device memory.  Structs
 *    passed by pointer (cgs_batch, cgs_scene, cgs_camera, cgs_scene_grads)
 *    live in host memory and are read during the call only.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and
 *    the call returns without synchronising.  No host<->device copies are
 *    made, so calls may be captured into a HIP graph.  cgs_render_forward
 *    and cgs_render_backward fork independent parts of their work (a scan, a
 *    sort by codebook row) to a second stream the library creates per device
 *    on first use (default priority, kept until the process ends) and join
 *    them back by events before returning: the caller's stream orders all of
 *    it, and a capture of that stream takes both.  The first call on a
 *    device should not be inside a capture (the second stream is not created
 *    then and the work stays on the caller's stream).
 *  - The return value covers host-side validation only (null pointers,
 *    negative sizes, unsupported options, workspace too small, launch
 *    failure).  Conditions found on the device are written to the caller's
 *    device array `d_info` (int64[4]): d_info[0] = status (CGS_OK or
 *    CGS_ECAPACITY), d_info[1] = number of (tile, Gaussian) instances the
 *    view batch needed.  Read it when convenient.
 *  - Gradients are overwritten, never accumulated.
 *  - Floating-point results are FP32; codebooks may be stored in FP32 or BF16.
 *  - All entry points are thread-compatible: concurrent calls must use
 *    different workspaces.
 *  - State the library keeps between calls (nothing else is global): per
 *    device, the second stream and its two events described above (created
 *    on first use, kept until the process ends; calls that fork to it are
 *    serialised per device by a mutex from fork to join, and an error return
 *    after the fork still joins it); a device counter of radix-sort waits
 *    that reached their bound (cgs_sort_stalls); per host thread, a scratch
 *    copy of the last batch plan (host memory, rebuilt by every call).
 */
#ifndef CGS_H
#define CGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CGS_OK = 0,
    CGS_EINVAL = -1,        /* bad argument (null pointer, negative size, bad stride, ...) */
    CGS_EUNSUPPORTED = -2,  /* valid but not supported by the library (e.g. sh_degree > 3) */
    CGS_ECAPACITY = -3,     /* instance capacity too small (device-side, via d_info) */
    CGS_EHIP = -4,          /* a HIP launch failed */
    CGS_EWORKSPACE = -5,    /* workspace too small */
    CGS_ELIMIT = -6         /* sizes beyond the fixed scratch of cgs_codebook_grad_reduce_noalloc */
} cgs_status;

typedef enum { CGS_F32 = 0, CGS_BF16 = 1 } cgs_dtype;

enum { CGS_MAX_VIEWS = 64, CGS_MAX_SCENES = 64, CGS_TILE = 16 };

/* Pinhole camera (the "camera pose P" of Sec. 2.1 / 4.2).  OpenCV axes:
 * x right, y down, z forward.  Pixel (x, y) samples image-plane point (x, y).
 * Rt: world->camera rotation and translation, row-major 3x4 [R | t].
 * campos: camera centre in world space (direction of view-dependent colour).
 * bg: background colour added with the final transmittance. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float Rt[12];
    float campos[3];
    float bg[3];
} cgs_camera;

/* A column window into a codebook (device memory, row-major).  Element (r, c)
 * of the window is ptr[r * row_stride + col0 + c] of type dtype. */
typedef struct {
    const void* ptr;
    int32_t dtype;       /* cgs_dtype */
    int32_t row_stride;  /* elements between consecutive rows */
    int64_t rows;        /* codebook size |SR| or |SH| */
    int32_t col0;
    int32_t pad_;
} cgs_cb_view;

/* One scene S = {G, C} (Sec. 4.1).
 * SR window columns: log-scale[3], quaternion (w,x,y,z)[4]; with
 *   opacity_mode == 1 column 7 of the SR window is the opacity logit.
 * SH window columns: 3 (sh_degree+1)^2 coefficients, coefficient-major and
 *   RGB-minor (c[j*3 + ch], j = l*l + l + m, real orthonormal harmonics with
 *   the Condon-Shortley phase).
 * Fused single-codebook layout [ls3 q4 logit1 sh...] with one index: idx_sr ==
 *   idx_sh, both windows on the same array, sr.col0 = 0, sh.col0 = 8,
 *   opacity_mode = 1.  The paper's two-codebook layout: separate windows and
 *   index arrays, per-Gaussian opacity (opacity_mode = 0). */
typedef struct {
    int64_t n;                    /* number of Gaussians (>= 0) */
    int32_t sh_degree;            /* 0..3, the same for every scene of a batch */
    int32_t opacity_mode;         /* 0: opacity_logit array, 1: SR window column 7 */
    const float* means;           /* device [n,3] */
    const int32_t* idx_sr;        /* device [n], values in [0, sr.rows) */
    const int32_t* idx_sh;        /* device [n], values in [0, sh.rows) */
    cgs_cb_view sr;
    cgs_cb_view sh;
    const float* opacity_logit;   /* device [n] when opacity_mode == 0, else NULL */
} cgs_scene;

/* Gradient outputs of one scene (device memory, FP32, overwritten).
 * sr / sh use the same window geometry as the scene's codebook windows
 * (rows x row_stride arrays, the window's columns written, others untouched).
 * opacity: [n] when opacity_mode == 0 (else unused). */
typedef struct {
    float* means;                 /* [n,3] */
    float* sr; int32_t sr_stride; int32_t sr_col0;
    float* sh; int32_t sh_stride; int32_t sh_col0;
    float* opacity;
} cgs_scene_grads;

/* Launch schedule knobs and optional instrumentation; zero-initialised
 * fields take the defaults.
 * stage_events: host array [CGS_STAGE_EVENTS] of hipEvent_t (caller-created)
 *   or NULL.  When set, the forward records event 0 before its first launch,
 *   1 after preprocessing, 2 after binning, 3 after the blend; the backward
 *   records 4 just before the backward blend, 5 after it, 6 after the
 *   per-Gaussian chain rule, 7 after the codebook reduction.  All on `stream`.
 * n_blend: device int32 [P] or NULL; when set the forward also writes the
 *   number of Gaussians blended into each pixel (a slower instrumented blend).
 * The schedule changes only the order work is issued in, never a result; the
 * backward must be given the same tile_order as the forward whose workspace it
 * reads (order 2 reuses the tile permutation the forward left there). */
enum { CGS_STAGE_EVENTS = 8 };
typedef struct {
    int32_t blend_waves_per_block;   /* waves (one 16x16 tile each) per workgroup: 1 (default), 2 or 4 */
    int32_t tile_order;              /* 0: row-major tiles, 1: XCD-grouped, 2: heaviest tile lists first */
    int32_t persistent;              /* 1: the blends run as a resident grid whose wavefronts take tiles from a
                                        queue in tile order (0 and 1 then both mean row-major), one wave per
                                        workgroup; 0 (default): one workgroup per group of tiles */
    int32_t reserved;
    void** stage_events;
    int32_t* n_blend;
} cgs_schedule;

/* A batch of views over one or more scenes, rendered by one call. */
typedef struct {
    const cgs_scene* scenes;      /* host array [n_scenes] */
    int32_t n_scenes;             /* 1..CGS_MAX_SCENES */
    int32_t n_views;              /* 1..CGS_MAX_VIEWS */
    const cgs_camera* cameras;    /* host array [n_views] */
    const int32_t* view_scene;    /* host array [n_views]: scene rendered by each view */
    int64_t instance_capacity;    /* max (tile, Gaussian) instances over the batch */
    const cgs_schedule* schedule; /* may be NULL */
} cgs_batch;

/* Images of a batch are stored view after view: view v occupies
 * [pix_off(v), pix_off(v) + H_v W_v) pixels, pix_off(v) = sum of earlier
 * views' H W; colour arrays are [pixels, 3] (RGB innermost). */

/* Workspace bytes needed by render_forward/render_backward for this batch
 * (the forward's binning results live in it until the backward).  Returns 0
 * for an invalid batch. */
size_t cgs_workspace_bytes(const cgs_batch* batch);

/* Forward render (Sec. 2.1 Eq. 1-3 over codebook-decoded Gaussians,
 * Sec. 4.2's I_P(G, C)).  For every Gaussian and view: gather its codebook
 * rows, scale = exp(log-scale), unit quaternion, opacity = sigmoid(logit);
 * project mean and covariance Sigma = R S S^T R^T (Eq. 2) with the
 * perspective Jacobian (Sigma2D = J W Sigma W^T J^T + 0.3 I); evaluate the
 * view-dependent SH colour max(0, sum Y_lm k_lm + 1/2); bin into 16x16 tiles
 * by (tile, depth, index); composite front to back per pixel (Eq. 3) with
 * alpha = min(0.99, o exp(power)), alpha < 1/255 skipped, stop before the
 * Gaussian that would take transmittance below 1e-4.
 * Outputs (device): image [P,3], T_final [P] (transmittance left after the
 * last blended Gaussian), n_last [P] (list position of the last blended
 * Gaussian + 1 in the pixel's tile list).  Workspace: >= cgs_workspace_bytes. */
cgs_status cgs_render_forward(const cgs_batch* batch, float* image, float* T_final, int32_t* n_last,
                              void* ws, size_t ws_bytes, int64_t* d_info, void* stream);

/* Backward of the forward render for dL/dimage = grad_image [P,3] (device).
 * Must follow cgs_render_forward on the same batch, workspace and outputs
 * (T_final, n_last as the forward wrote them; the per-pixel transmittance of
 * every blended Gaussian is recomputed from T_final by division, not stored;
 * the codebook indices unchanged since the forward, which also ordered the
 * Gaussians by codebook row for this call).
 * Writes, per scene, dL/dmeans and dL/dcodebook: the per-Gaussian parameter
 * gradients summed over Gaussians sharing a codebook row (the gradient of
 * S_diff needed by the update step, Sec. 4.4).  Deterministic: every sum is
 * taken in a fixed order (no floating-point atomics), so repeated calls give
 * bitwise-identical gradients.  grads: host array [n_scenes]. */
cgs_status cgs_render_backward(const cgs_batch* batch, const float* grad_image,
                               const float* T_final, const int32_t* n_last,
                               const cgs_scene_grads* grads,
                               void* ws, size_t ws_bytes, int64_t* d_info, void* stream);

/* SGLD step sizes and noise stream of the parameter-update transition
 * (Sec. 2.3's SGLD rule; Sec. 4.4 and App. A.1: theta' = theta + (eps/2)
 * grad log p + sqrt(eps) eta with log p = -L, one eps per parameter kind).
 * eps_* >= 0 (0 leaves that kind unchanged); eta ~ N(0, 1) from the
 * counter-based generator described at cgs_sgld_normals, keyed by `seed`,
 * `step` selecting the stream of one training step. */
typedef struct {
    float eps_means, eps_opacity, eps_sr, eps_sh;
    uint64_t seed;
    uint32_t step;
    uint32_t pad_;
} cgs_sgld;

/* FP32 parameters an SGLD update writes, per scene (device pointers):
 * means [n,3]; opacity_logit [n] (opacity_mode 0, else NULL); sr: rows whose
 * columns sr_col0 .. hold ls3 q4 (and the opacity logit when opacity_mode is
 * 1); sh: rows whose columns sh_col0 .. hold the 3(d+1)^2 SH coefficients.
 * They may be the scene's own FP32 arrays (updated in place); otherwise the
 * scene's arrays the renderer reads are refreshed from the updated values
 * (BF16 codebooks by round-to-nearest-even). */
typedef struct {
    float* means;
    float* opacity_logit;
    float* sr; int32_t sr_stride; int32_t sr_col0;
    float* sh; int32_t sh_stride; int32_t sh_col0;
} cgs_scene_params;

/* cgs_render_backward followed by one SGLD step of every parameter, fused
 * into the chain-rule epilogue (means, per-Gaussian opacity) and the codebook
 * reduction epilogue (codebook rows, rows no Gaussian maps to included), so
 * neither the gradients nor the parameters make another pass through HBM:
 *   theta <- theta - (eps/2) dL/dtheta + sqrt(eps) eta.
 * Gradients are still written to `grads`.  Step sizes per row-layout column:
 * ls and q eps_sr, the logit eps_opacity, SH eps_sh.  Noise streams (see
 * cgs_sgld_normals): Gaussian g of scene s uses counter index g, tag
 * 0x10000 s, normals 0-2 for the mean and 3 for the per-Gaussian logit;
 * codebook row k, row-layout column c uses index 16 k + c / 4, tag
 * 0x10000 s + 1, normal c % 4.  The parameters must not alias the gradient
 * buffers.  params: host array [n_scenes].  Deterministic. */
cgs_status cgs_render_backward_sgld(const cgs_batch* batch, const float* grad_image, const float* T_final,
                                    const int32_t* n_last, const cgs_scene_grads* grads, const cgs_sgld* sgld,
                                    const cgs_scene_params* params, void* ws, size_t ws_bytes, int64_t* d_info,
                                    void* stream);

/* The SGLD noise generator on its own: for i < n, counter (index0 + i as
 * 64-bit lo, hi; tag; step) under key seed (lo, hi) through Philox4x32-10
 * (Salmon et al., SC 2011); words [n][4] (device, may be NULL) receive the raw
 * output, z [n][4] (device) the Box-Muller normals of the pairs (w0, w1) and
 * (w2, w3): u = ((w >> 9) + 1/2) 2^-23, z = sqrt(-2 ln u_a) (cos, sin)(2 pi u_b). */
cgs_status cgs_sgld_normals(int64_t n, uint64_t index0, uint32_t tag, uint32_t step, uint64_t seed, float* z,
                            uint32_t* words, void* stream);

/* Reconstruction loss of Eq. 4 over a batch of views and its gradient:
 * L = (1 - lambda) L1 + lambda (1 - mean SSIM), both means over every pixel
 * and channel of the batch.  SSIM (Wang et al. 2004): 11x11 Gaussian window
 * of sigma 1.5 (normalised), C1 = 0.01^2, C2 = 0.03^2, local statistics by
 * same-size convolution with zero padding, per channel.  image, target, grad:
 * device [P,3] in the renderer's layout (views concatenated, row-major);
 * hw: host int32 [n_views][2] (height, width); loss: device float[1]; grad is
 * written.  0 <= lambda <= 1.  Workspace: cgs_loss_recon_workspace_bytes. */
size_t cgs_loss_recon_workspace_bytes(int32_t n_views, const int32_t* hw);

/* Metropolis-Hastings moves on a codebook (the split and merge transitions of
 * the proposal mixture, Sec. 4.4 and App. A.1).  One call makes n_proposals
 * independent proposals from counter-based Philox streams (counter 16 b + j,
 * tag 0x20000 split / 0x20001 merge, `step`, key `seed`).
 * Split: Gaussian g = floor(w0 n / 2^32), offset u ~ N(0, eps_split^2 I) over
 * the row, accepted with the paper's probability min(1, e^-lambda / q_sm(u)),
 * q_sm(u) = exp(-|u|^2/2 (1/eps_split^2 - 1/eps_merge^2)); a Gaussian splits
 * at most once per call (lowest proposal); accepted splits in proposal order
 * append rows c + u (row c keeps its value) while rows < K_max and move g.
 * Merge: a uniform pair of distinct live rows (c, c'), thinned by
 * exp(-|c - c'|^2 / (2 eps_merge^2)) so that selected pairs follow q_merge,
 * accepted with min(1, e^lambda q_sm(c - c')); a row joins at most one merge
 * per call (later proposals naming it are withdrawn); the Gaussians of c'
 * move to c, and live rows are compacted to 0 .. K'-1 (freed rows below K'
 * take the surviving rows above, ascending).
 * Deterministic (integer atomics only).  lambda is the prior cost of a row of
 * this codebook (lambda_SR or lambda_SH). */
typedef struct {
    float lambda, eps_split, eps_merge;
    int32_t n_proposals;
    uint64_t seed;
    uint32_t step;
    uint32_t pad_;
} cgs_mh;

/* The codebook the moves act on (device pointers): FP32 rows [K_max, ld]
 * holding D <= 60 values each from column 0; d_rows: device int64, the live
 * row count K (read and updated on the device); idx [n] int32 row of each
 * Gaussian; mirror: optional BF16 copy [K_max, mirror_ld] the renderer reads
 * (rows written by a move are refreshed by round-to-nearest-even) or NULL. */
typedef struct {
    float* rows; int64_t ld; int64_t D; int64_t K_max;
    int64_t* d_rows;
    int32_t* idx; int64_t n;
    uint16_t* mirror; int64_t mirror_ld;
} cgs_mh_codebook;

size_t cgs_mh_workspace_bytes(const cgs_mh_codebook* cb, int32_t n_proposals);
cgs_status cgs_mh_split(const cgs_mh_codebook* cb, const cgs_mh* p, void* ws, size_t ws_bytes, void* stream);
cgs_status cgs_mh_merge(const cgs_mh_codebook* cb, const cgs_mh* p, void* ws, size_t ws_bytes, void* stream);

/* Host only: the transition a training step takes under the proposal mixture
 * (0 parameter update, 1 split, 2 merge with probabilities 0.98 / 0.01 /
 * 0.01), from uniform24 of word 0 of Philox counter (0, 0, 0x20002, step). */
int32_t cgs_mh_transition(uint64_t seed, uint32_t step);
cgs_status cgs_loss_recon(const float* image, const float* target, int32_t n_views, const int32_t* hw,
                          float lambda_ssim, float* grad, float* loss, void* ws, size_t ws_bytes, void* stream);

/* Codebook gradient reduction (Sec. 2.2 / 4.1: a Gaussian's parameters are
 * its codebook row, so a row's gradient is the sum over the Gaussians mapped
 * to it): grad_cb[k, c] = sum_{i : idx[i] == k} g[i * ld + c], c < d.
 * g: device [n, ld] FP32; idx: device [n] in [0, k); perm: device [n]
 * Gaussian indices stably sorted by idx (cached by the caller while the
 * indices do not change) or NULL to sort here; grad_cb: device [k, ld_out],
 * columns [0, d) overwritten (rows with no Gaussian get 0).  Order-fixed and
 * deterministic.  Workspace: cgs_codebook_grad_reduce_workspace_bytes. */
size_t cgs_codebook_grad_reduce_workspace_bytes(int64_t n, int64_t k, int32_t d);
cgs_status cgs_codebook_grad_reduce(const float* g, int64_t ld, const int32_t* idx, const int32_t* perm,
                                    int64_t n, int64_t k, int32_t d, float* grad_cb, int64_t ld_out,
                                    void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reduction as cgs_codebook_grad_reduce, same arguments and the same kernels
 * (so the same bits), with its workspace taken from a scratch array the
 * library holds in device memory instead of a caller workspace.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * Limit: cgs_codebook_grad_reduce_workspace_bytes(n, k, d) must not exceed
 * 32 MiB (about n = 1.9M Gaussians at k = 65536 rows); larger sizes return
 * CGS_ELIMIT before any launch.  The scratch is one array per device, taken
 * when the library is loaded there and held until the process ends; its
 * address is looked up on the first call on each device (with that device
 * current), which may return CGS_EHIP if the lookup fails.  Every call on a
 * device shares that device's array and the array keeps what the last call
 * left in it (everything the reduction needs zeroed it clears itself), so
 * calls that overlap in time on one device -- on different streams or from
 * different host threads -- race and must not be issued. */
cgs_status cgs_codebook_grad_reduce_noalloc(const float* g, int64_t ld, const int32_t* idx, const int32_t* perm,
                                            int64_t n, int64_t k, int32_t d, float* grad_cb, int64_t ld_out,
                                            void* stream);

/* Tile binning of the 3DGS tile renderer the paper builds on (Sec. 2.1):
 * every (Gaussian i, tile t in its rectangle) instance gets the key
 * ((view_of[i] * tiles_y + ty) * tiles_x + tx) << 32 | depth_key[i]; instances
 * are emitted in Gaussian order (tiles row-major) and stably sorted by key.
 * depth_key: device [n] (IEEE bits of positive view depths); trect: device
 * [n,4] uint16 half-open tile rectangle x0,y0,x1,y1 (empty = no instance);
 * view_of: device [n] or NULL (all view 0).  Outputs (device): sorted_key
 * [capacity] (may be NULL), sorted_gid [capacity], tile_range
 * [n_views*tiles_y*tiles_x, 2] = half-open [start, end) of each tile (start =
 * end for an empty tile).  If the instance count exceeds capacity nothing is
 * sorted and d_info[0] = CGS_ECAPACITY; d_info[1] = instance count. */
size_t cgs_bin_tiles_workspace_bytes(int64_t n, int32_t tiles_x, int32_t tiles_y, int32_t n_views,
                                     int64_t capacity);
cgs_status cgs_bin_tiles(const uint32_t* depth_key, const uint16_t* trect, const int32_t* view_of,
                         int64_t n, int32_t tiles_x, int32_t tiles_y, int32_t n_views,
                         uint64_t* sorted_key, uint32_t* sorted_gid, uint32_t* tile_range,
                         int64_t capacity, int64_t* d_info, void* ws, size_t ws_bytes, void* stream);

/* L1 part of the reconstruction loss (Sec. 2.1 Eq. 4 with the SSIM weight 0):
 * loss = mean |image - target| over n values, grad = sign(image - target) / n
 * (sign(0) = 0).  image, target, grad: device [n]; loss: device float[1]
 * (written, not accumulated).  Workspace: cgs_loss_l1_workspace_bytes(n). */
size_t cgs_loss_l1_workspace_bytes(int64_t n);
cgs_status cgs_loss_l1(const float* image, const float* target, int64_t n, float* grad, float* loss,
                       void* ws, size_t ws_bytes, void* stream);

/* Offsets (bytes from the workspace base) of the forward's intermediate
 * arrays for a batch, for inspection and tests.  Any pointer may be NULL.
 * records: R = sum over views of the view's scene size, record r of view v is
 *   Gaussian r - rec_off(v) of that scene; records float4 [R][3], 48 B each:
 *   (u, v, -A/2 L, -B L), (-C/2 L, opacity, red, green), (blue, tile_rect[0]
 *   bits, tile_rect[1] bits, o) -- A, B, C the conic (inverse of
 *   Sigma2D), L = log2(e), o (uint32 bits) the offset of the record's first
 *   backward gradient slot within its 64-record chunk; depth_key uint32 [R]
 *   (0x7f800000 when culled);
 *   tile_rect uint32[R][2] ((x0 | y0 << 16), (x1 | y1 << 16)), written only
 *   when some view of the batch is 256 tiles or more across or down (below
 *   that the rectangle travels packed in one word); the same two words are
 *   always words 9 and 10 of the record (zero when culled);
 * inst_rec uint32 [capacity] record of each sorted instance; tile_range
 *   uint32 [tiles][2]. */
typedef struct {
    size_t records, depth_key, tile_rect, inst_rec, tile_range;
    int64_t n_records, n_tiles;
} cgs_ws_layout;
cgs_status cgs_workspace_layout(const cgs_batch* batch, cgs_ws_layout* out);

/* Human-readable name of a status code (static string). */
const char* cgs_status_str(int32_t status);

/* Library version: major*10000 + minor*100 + patch. */
int32_t cgs_version(void);

/* Diagnostic of the radix sorts inside the binning, the codebook reduction
 * and cgs_bin_tiles: the number of look-back waits that reached their bound on
 * the current device since the library was loaded.  A sorting workgroup
 * waits only on workgroups that started before it and publish their counts
 * without waiting, so this stays 0; a nonzero value means that the sorted
 * output of some call since then is wrong (its writes stay in bounds).
 * Synchronous (a device read on the null stream); 0xffffffff if that read
 * fails. */
uint32_t cgs_sort_stalls(void);

#ifdef __cplusplus
}
#endif

#endif /* CGS_H */
