// Backward render: reverse-order blend (transmittance recovered from T_final
// by division), per-Gaussian chain rule from the projected parameters to the
// mean and the codebook-row values, and the codebook reduction as a sort by
// row index followed by fixed-order segmented sums (no contended atomics).
#include "cgs_internal.h"
#include "philox.h"
#include "render_common.h"
#include "wave_scan.h"

namespace cgs {

// ------------------------------------------------------------ backward blend
// One wavefront per tile, same pixel mapping and quadrant skipping as the
// forward (with the quadrant masks the forward stored per list position).
// Each pixel walks its list from n_last-1 down to 0, re-derives alpha with
// the forward's code, recovers T before the Gaussian as
// T_after / (1 - alpha), and accumulates dL/d(u, v, -A/2, -B, -C/2, opacity,
// r, g, b).  The lane's four pixels are summed in registers, then over the
// wave by DPP row shifts and row broadcasts into lane 63, which parks the
// record's nine sums in LDS for the lane that loaded the record.  The tile's total for a record
// goes to that (tile, record) instance's own slot -- the record's slot offset
// (tile counts scanned in record order) + the tile's row-major index in the
// record's rectangle -- with plain
// stores: no atomics, and the per-record sum over its tiles is taken later in
// a fixed order, so the backward is deterministic.  Instances the walk never
// reaches (beyond every pixel's n_last) are not touched: the tile's cut,
// written here, tells the chain-rule kernel which slots hold values.
//
// PERSIST: the grid is resident and each wavefront takes tiles from the
// backward's tile queue until it runs dry (same per-tile work and results).
template <int WPB, bool PERSIST>
__global__ __launch_bounds__(WPB * 64) void k_blend_bwd(const BatchDesc* __restrict__ desc,
                                                         const uint32_t* __restrict__ ranges,
                                                         const uint32_t* __restrict__ inst_rec,
                                                         const float4* __restrict__ rec,
                                                         const uint8_t* __restrict__ qbits,
                                                         const uint32_t* __restrict__ depth_key,
                                                         const uint32_t* __restrict__ chunk_base,
                                                         const float* __restrict__ grad_image,
                                                         const float* __restrict__ T_final,
                                                         const int32_t* __restrict__ n_last,
                                                         float* __restrict__ ginst, uint2* __restrict__ tile_cut,
                                                         DevCounters* __restrict__ cnt) {
    __shared__ float4 s_g[WPB][64];
    __shared__ float4 s_c[WPB][64];
    __shared__ float s_b[WPB][64];
    __shared__ uint32_t s_p[WPB][64];
    __shared__ uint32_t s_s[WPB][64];                          // gradient slot of each staged record
    __shared__ __align__(16) float s_red[WPB][2][9][64];        // per-lane sums of a pair of records, by value
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t fetched = 0u;
    if constexpr (PERSIST) fetched = fetch_pos(cnt->q_bwd, lane);
    for (int it = 0;; ++it) {
        int64_t tile;
        if constexpr (PERSIST) {
            tile = tile_at(desc, fetched);
            if (tile < desc->n_tiles) fetched = fetch_pos(cnt->q_bwd, lane);   // the next one, waited for at the top
        } else {
            if (it > 0) break;
            tile = __builtin_amdgcn_readfirstlane((int)tile_index(desc, blockIdx.x, gridDim.x, w, WPB));
        }
        if (tile >= desc->n_tiles) break;
        const int v = find_view_by_tile(desc, tile);
        const ViewDesc& vd = desc->views[v];
        const int64_t lt = tile - vd.tile_off;
        const int tx = (int)(lt % vd.tiles_x), ty = (int)(lt / vd.tiles_x);
        const int x0 = tx * kTile, y0 = ty * kTile;

        // Bh[k]: dL/dC . (colour composited behind the current position,
        // normalised to unit transmittance), starting from the background --
        // dL/dC is fixed per pixel, so one scalar replaces the three channels
        float T[4], dC0[4], dC1[4], dC2[4], Bh[4], fpx[4], fpy[4];
        uint32_t last[4];
        uint32_t maxlast = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int px = x0 + 8 * (k & 1) + (lane & 7), py = y0 + 8 * (k >> 1) + (lane >> 3);
            fpx[k] = (float)px;
            fpy[k] = (float)py;
            if (px < vd.W && py < vd.H) {
                const int64_t p = vd.pix_off + (int64_t)py * vd.W + px;
                T[k] = T_final[p];
                last[k] = (uint32_t)n_last[p];
                dC0[k] = grad_image[3 * p + 0];
                dC1[k] = grad_image[3 * p + 1];
                dC2[k] = grad_image[3 * p + 2];
            } else {
                T[k] = 1.f; last[k] = 0; dC0[k] = dC1[k] = dC2[k] = 0.f;
            }
            Bh[k] = fmaf(dC0[k], vd.bg[0], fmaf(dC1[k], vd.bg[1], dC2[k] * vd.bg[2]));
            maxlast = last[k] > maxlast ? last[k] : maxlast;
        }
        maxlast = wave_max_u32(maxlast);
        const uint32_t start = ranges[2 * tile];
        const uint32_t len = ranges[2 * tile + 1] - start;
        if (maxlast > len) maxlast = len;     // n_last inconsistent with this binning: stay in the list
        // The walk covers list positions [0, maxlast).  Lists are ordered by
        // (depth key, record), so the first position it does not reach is named
        // by that pair; the chain-rule kernel reads only slots ordered before it
        // and the slots beyond are never written.
        if (lane == 0) {
            uint2 cut = make_uint2(0xffffffffu, 0xffffffffu);
            if (maxlast < len) {
                const uint32_t c = inst_rec[start + maxlast];
                cut = make_uint2(depth_key[c], c);
            }
            tile_cut[tile] = cut;
        }
        for (int64_t bend = maxlast; bend > 0; bend -= 64) {
            const int64_t bbeg = bend - 64 > 0 ? bend - 64 : 0;
            const int64_t li = bbeg + lane;
            int64_t slot = -1;
            uint32_t qm = 0u;
            float4 g, c;
            float bl = 0.f;
            if (li < bend) {
                const uint32_t r = inst_rec[start + li];
                g = rec[kRecF4 * (int64_t)r + 0];
                c = rec[kRecF4 * (int64_t)r + 1];
                const float4 x = rec[kRecF4 * (int64_t)r + 2];
                bl = x.x;
                const uint32_t rlo = __float_as_uint(x.y), rhi = __float_as_uint(x.z);
                const int rx0 = (int)(rlo & 0xffffu), ry0 = (int)(rlo >> 16), rx1 = (int)(rhi & 0xffffu);
                // the record's slots: its chunk's base (a small table, cached) +
                // its offset in the chunk (the record's spare word) + the tile's
                // row-major index in the record's rectangle
                const uint32_t cb = chunk_base[vd.rec_wave_off + ((int64_t)(r - (uint32_t)vd.rec_off) >> 6)];
                slot = (int64_t)cb + __float_as_uint(x.w) + (int64_t)(ty - ry0) * (rx1 - rx0) + (tx - rx0);
                qm = qbits[start + li];     // the forward's quadrant mask of this record
            }
            const uint64_t km = __ballot(qm != 0u);
            const uint32_t mine = popc_below(km);
            if (qm != 0u) {
                s_g[w][mine] = g;
                s_c[w][mine] = c;
                s_b[w][mine] = bl;
                s_p[w][mine] = ((uint32_t)li << 4) | qm;
                s_s[w][mine] = (uint32_t)slot;
            }
            wave_sync();
            const int cnt = (int)__popcll(km);
            for (int j = cnt - 1; j >= 0; --j) {
                const uint32_t pq = __builtin_amdgcn_readfirstlane(s_p[w][j]);
                const uint32_t pos = pq >> 4;     // 0-based list position
                const float4 gg = s_g[w][j];
                const float4 cc = s_c[w][j];
                const float bb = s_b[w][j];
                float a_u = 0.f, a_v = 0.f, a_a = 0.f, a_b = 0.f, a_c = 0.f, a_o = 0.f, a_r = 0.f, a_g = 0.f, a_bl = 0.f;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (!((pq >> k) & 1u)) continue;          // wave-uniform quadrant skip
                    const float dx = fpx[k] - gg.x;
                    const float dy = fpy[k] - gg.y;
                    float G;
                    bool pcl;
                    const float alpha = blend_alpha(dx, dy, gg, cc, G, pcl);
                    const bool use = (pos < last[k]) && (alpha >= kMinAlpha);
                    if (__ballot(use) == 0ull) continue;       // no pixel of the quadrant blended it
                    // Branch-free for the lanes of the quadrant: pairs the forward
                    // did not blend get alpha 0 and zero gradients, which leaves T
                    // and the background sum unchanged.
                    // (rcp(1) = 1 exactly, so an unused pair leaves T as it is)
                    const float am = use ? alpha : 0.f;
                    const float Tb = T[k] * __builtin_amdgcn_rcpf(1.f - am);
                    const float wgt = am * Tb;
                    a_r = fmaf(wgt, dC0[k], a_r);
                    a_g = fmaf(wgt, dC1[k], a_g);
                    a_bl = fmaf(wgt, dC2[k], a_bl);
                    // dL/dalpha = T_before (dL/dC . c - Bh); Bh <- Bh + alpha (dL/dC . c - Bh)
                    const float e = fmaf(dC0[k], cc.z, fmaf(dC1[k], cc.w, dC2[k] * bb)) - Bh[k];
                    const float dal = Tb * e;
                    Bh[k] = fmaf(am, e, Bh[k]);
                    T[k] = Tb;
                    const bool open = use && (alpha < kMaxAlpha);      // alpha not saturated at 0.99
                    const float dao = open ? dal : 0.f;
                    a_o = fmaf(dao, G, a_o);
                    const float dp = (open && !pcl) ? dal * alpha : 0.f;  // dL/dpower
                    const float dpx = dp * dx, dpy = dp * dy;
                    a_a = fmaf(dpx, dx, a_a);
                    a_b = fmaf(dpx, dy, a_b);
                    a_c = fmaf(dpy, dy, a_c);
                    // dL/du = -(2 a' Sx + b' Sy), dL/dv = -(2 c' Sy + b' Sx) with
                    // Sx = sum dp dx, Sy = sum dp dy (a' = -A/2, b' = -B, c' = -C/2);
                    // the conic is the record's, so the sums are taken first.
                    a_u += dpx;
                    a_v += dpy;
                }
                // This lane's nine sums for record j, the position sums already
                // turned into dL/du, dL/dv by the record's natural-log conic (a
                // linear map, so it is applied before the sum over lanes).
                {
                    const float na2 = 2.f * kLn2 * gg.z, nb = kLn2 * gg.w, nc2 = 2.f * kLn2 * cc.x;
                    float* red = &s_red[w][j & 1][0][lane];
                    red[0 * 64] = -fmaf(na2, a_u, nb * a_v);
                    red[1 * 64] = -fmaf(nc2, a_v, nb * a_u);
                    red[2 * 64] = a_a;
                    red[3 * 64] = a_b;
                    red[4 * 64] = a_c;
                    red[5 * 64] = a_o;
                    red[6 * 64] = a_r;
                    red[7 * 64] = a_g;
                    red[8 * 64] = a_bl;
                }
                if ((j & 1) == 0) {
                    // Sum the pair (records j, j + 1 if staged) over the lanes: the
                    // 2 x 9 value vectors are split into 8-lane segments; lane l of
                    // round t takes segment l & 7 of vector (64 t + l) >> 3, adds its
                    // eight values, the segments of a vector are combined by DPP row
                    // shifts into its last lane, which writes the record's slot.
                    wave_sync();
                    const int nrec = cnt - j < 2 ? cnt - j : 2;
#pragma unroll
                    for (int t = 0; t < 3; ++t) {
                        const int p = 64 * t + lane;
                        const int rec = p >= 72 ? 1 : 0;
                        const int val = (p - 72 * rec) >> 3;
                        const bool ok = p < 144 && rec < nrec;
                        float x = 0.f;
                        if (ok) {
                            const float4 lo = *reinterpret_cast<const float4*>(&s_red[w][rec][val][8 * (lane & 7)]);
                            const float4 hi = *reinterpret_cast<const float4*>(&s_red[w][rec][val][8 * (lane & 7) + 4]);
                            x = ((lo.x + lo.y) + (lo.z + lo.w)) + ((hi.x + hi.y) + (hi.z + hi.w));
                        }
                        x = group8_sum_to_last(x);
                        if (ok && (lane & 7) == 7) ginst[9 * (int64_t)s_s[w][j + rec] + val] = x;
                    }
                    wave_sync();
                }
            }
            wave_sync();
            if (slot >= 0 && qm == 0u) {       // a record no pixel of the tile blended
                float* dst = ginst + 9 * slot;
#pragma unroll
                for (int k = 0; k < 9; ++k) dst[k] = 0.f;
            }
            wave_sync();
        }
    }
    if constexpr (PERSIST) retire_wave(cnt->q_bwd, &cnt->done_bwd, (unsigned long long)gridDim.x * WPB, lane);
}

// ------------------------------------------------------- record gradients
// dL/d(record) for every (view, Gaussian) record = the sum of the record's
// tile slots, in row-major tile order, over the tiles whose backward walk
// reached the record -- (depth key, record) ordered before the tile's cut.
// Written as 9 floats per record, only for records with a nonzero sum; a bit
// per record says which, so records no walk reached cost neither a write nor
// a read.  The bits of wavefront f (64 records of one view; a scene's views of
// the same 64 Gaussians side by side, f = flag_wave_off + q vcount + vi) are
// words 8 f and 8 f + 4, next to the forward's colour-clamp bits of the same
// records (words 8 f + 4 h + 1..3), so the chain rule reads all four of a
// record's flags with one 16-byte load.
//
// Wave-cooperative: a wavefront owns 64 consecutive records, whose slots are
// one contiguous range.  The lanes walk that range 64 slots at a time, one
// slot each (its record by a max-scan of per-record start marks),
// so a record covering many tiles does not hold up the other 63; only the
// slots the walk reached are loaded, and each lane adds its own record's
// reached slots of the chunk from LDS in slot order -- the order, and so the
// bits, of a sequential sum per record (an unreached slot would add +0).

__global__ __launch_bounds__(256) void k_slot_sum(const BatchDesc* __restrict__ desc, const float* __restrict__ ginst,
                                                  const uint32_t* __restrict__ chunk_base,
                                                  const uint32_t* __restrict__ ntiles,
                                                  const uint2* __restrict__ tile_rect,
                                                  const uint32_t* __restrict__ prect,
                                                  const uint32_t* __restrict__ depth_key,
                                                  const uint2* __restrict__ tile_cut,
                                                  const DevCounters* __restrict__ cnt, float* __restrict__ rec_grad,
                                                  uint32_t* __restrict__ rec_flag, uint32_t* __restrict__ isl_flag,
                                                  int64_t n_isl) {
    __shared__ uint32_t s_start[4][64], s_so[4][64], s_key[4][64], s_org[4][64], s_w[4][64], s_mark[4][64];
    // the chain rule's island flag words start from zero
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_isl; i += (int64_t)gridDim.x * blockDim.x)
        isl_flag[i] = 0u;
    __shared__ float s_v[4][9][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t wv = wave_id(4);
    if (wv >= desc->n_rec_waves) return;
    const ViewDesc& vd = desc->views[find_view_by_wave(desc, wv)];
    const int64_t i0 = (wv - vd.rec_wave_off) * kWave;
    const int64_t i = i0 + lane;
    const bool valid = i < desc->scenes[vd.scene].n;
    // the record's words are loaded together (lanes past the end read the
    // wave's first record and own no slots); with every view below 256 tiles
    // per side the rectangle is one packed word (x0 | y0 << 8 | x1 << 16 |
    // y1 << 24, zero when culled) and the tile count follows from it
    const int64_t r = vd.rec_off + (valid ? i : i0);
    uint2 tr;
    uint32_t ntr;
    if (desc->pack_rect) {
        const uint32_t pr = prect[r];
        const uint32_t x0 = pr & 0xffu, y0 = (pr >> 8) & 0xffu, x1 = (pr >> 16) & 0xffu, y1 = pr >> 24;
        tr = make_uint2(x0 | (y0 << 16), x1 | (y1 << 16));
        ntr = (x1 - x0) * (y1 - y0);
    } else {
        tr = tile_rect[r];
        ntr = ntiles[r];
    }
    const uint32_t key = depth_key[r];
    const uint32_t nt = valid && cnt->n_inst_ok != 0ull ? ntr : 0u;
    const uint32_t incl = wave_incl_sum_u32(nt, lane);
    const uint32_t start = incl - nt;
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t so = chunk_base[wv] + start;     // the chunk's slots are contiguous
    float d[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (total != 0u) {
        s_start[w][lane] = start;
        s_so[w][lane] = so;
        s_key[w][lane] = key;
        s_org[w][lane] = tr.x;                                   // rx0 | ry0 << 16
        s_w[w][lane] = (tr.y & 0xffffu) - (tr.x & 0xffffu);      // rectangle width in tiles
        wave_sync();
        const uint2* cutv = tile_cut + vd.tile_off;
        const uint32_t rec0 = (uint32_t)(vd.rec_off + i0);
        const uint32_t my_end = start + nt;
        uint32_t carry = 0u;     // 1 + the lane of the record owning the last slot of the previous chunk
        for (uint32_t c0 = 0; c0 < total; c0 += 64) {
            // each record with slots marks the lane of its first slot in the
            // chunk; a max-scan of the marks gives every slot its record
            s_mark[w][lane] = 0u;
            wave_sync();
            if (nt > 0u && start >= c0 && start < c0 + 64u) s_mark[w][start - c0] = (uint32_t)lane + 1u;
            wave_sync();
            uint32_t mk = wave_incl_max_u32(s_mark[w][lane], lane);
            mk = mk > carry ? mk : carry;
            carry = (uint32_t)__builtin_amdgcn_readlane((int)mk, 63);
            const uint32_t k = c0 + (uint32_t)lane;
            bool reached = false;
            if (k < total) {
                // the last record of the wave whose slots start at or before k
                const int lo = (int)mk - 1;
                const uint32_t e = k - s_start[w][lo];
                const uint32_t wq = s_w[w][lo];
                // e / wq: the quotient is a row of the rectangle (< 2^16), so
                // the FP32 estimate is off by less than 1/64: one step each way
                uint32_t row = (uint32_t)((float)e * __builtin_amdgcn_rcpf((float)wq));
                row -= row * wq > e ? 1u : 0u;
                row += (row + 1) * wq <= e ? 1u : 0u;
                const uint32_t org = s_org[w][lo];
                const uint2 ct = cutv[(int64_t)((org >> 16) + row) * vd.tiles_x + (org & 0xffffu) + (e - row * wq)];
                const uint32_t kk = s_key[w][lo];
                // both words of the cut in one load (no short-circuit on ct.x)
                reached = (kk < ct.x) | ((kk == ct.x) & (rec0 + (uint32_t)lo < ct.y));
                if (reached) {
                    const float* src = ginst + 9 * ((int64_t)s_so[w][lo] + e);
#pragma unroll
                    for (int q = 0; q < 9; ++q) s_v[w][q][lane] = src[q];
                }
            }
            const uint64_t rm = __ballot(reached);
            wave_sync();
            // this lane's record's reached slots of the chunk, in slot order
            // (an unreached slot would add +0, which changes no nonzero sum)
            const uint32_t a = start > c0 ? start - c0 : 0u;
            const uint32_t b = my_end < c0 + 64u ? (my_end > c0 ? my_end - c0 : 0u) : 64u;
            uint64_t mm = 0ull;
            if (a < b) mm = rm & (b == 64u ? ~0ull : (1ull << b) - 1ull) & ~((1ull << a) - 1ull);
            while (mm) {
                const int j = (int)__builtin_ctzll(mm);
                mm &= mm - 1ull;
#pragma unroll
                for (int q = 0; q < 9; ++q) d[q] += s_v[w][q][j];
            }
            wave_sync();
        }
    }
    bool nz = false;
#pragma unroll
    for (int k = 0; k < 9; ++k) nz |= d[k] != 0.f;
    const uint64_t m = __ballot(nz);
    if (lane == 0) {
        const SceneDesc& sd = desc->scenes[vd.scene];
        const int64_t fw = sd.flag_wave_off + (wv - vd.rec_wave_off) * sd.vcount + vd.scene_vi;
        rec_flag[8 * fw] = (uint32_t)m;
        rec_flag[8 * fw + 4] = (uint32_t)(m >> 32);
    }
    if (nz) {
        float* out = rec_grad + 9 * r;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = d[k];
    }
}

// ------------------------------------------------------------ SGLD update
// theta <- theta - (eps/2) dL/dtheta + sqrt(eps) eta, eta ~ N(0, 1) from the
// Philox streams (the parameter-update transition: grad log p = -grad L).
// The FP32 master is updated in place and, when the renderer reads a
// different copy (BF16 codebook, separate FP32 array), that copy is refreshed
// from the new master (BF16 by round-to-nearest-even).

// A Gaussian's own parameters: mean, and the opacity logit when it is per
// Gaussian.
__device__ inline void sgld_gaussian(const BatchDesc* desc, const SceneDesc& sd, int s, int64_t g, const float dmu[3],
                                     float dlogit) {
    float z[4];
    normals4((uint64_t)g, gaussian_tag(s), (uint32_t)desc->step, desc->seed, z);
    if (sd.u_means) {
        const float e = desc->eps[0], h = 0.5f * e, r = sqrtf(e);
        float* mirror = const_cast<float*>(sd.means);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float v = sd.u_means[3 * g + k] - h * dmu[k] + r * z[k];
            sd.u_means[3 * g + k] = v;
            if (mirror != sd.u_means) mirror[3 * g + k] = v;
        }
    }
    if (sd.opacity_mode == 0 && sd.u_opacity) {
        const float e = desc->eps[1];
        const float v = sd.u_opacity[g] - 0.5f * e * dlogit + sqrtf(e) * z[3];
        sd.u_opacity[g] = v;
        float* mirror = const_cast<float*>(sd.opacity);
        if (mirror != sd.u_opacity) mirror[g] = v;
    }
}

// One codebook entry: row lr (scene-local) of scene s, row-layout column gc
// (ls 0-2, q 3-6, logit 7, SH 8-), with its reduced gradient.
__device__ inline void sgld_row(const BatchDesc* desc, int s, int64_t lr, int gc, float grad) {
    const SceneDesc& sd = desc->scenes[s];
    const bool srp = gc < 8;
    float* m = srp ? sd.u_sr : sd.u_sh;
    if (!m) return;
    m += srp ? lr * sd.u_sr_stride + sd.u_sr_col0 + gc : lr * sd.u_sh_stride + sd.u_sh_col0 + (gc - 8);
    const float e = gc < 7 ? desc->eps[2] : (gc == 7 ? desc->eps[1] : desc->eps[3]);
    float z[4];
    normals4(16u * (uint64_t)lr + (uint64_t)(gc >> 2), codebook_tag(s), (uint32_t)desc->step, desc->seed, z);
    const float v = *m - 0.5f * e * grad + sqrtf(e) * z[gc & 3];
    *m = v;
    const int64_t off = srp ? lr * sd.sr_stride + sd.sr_col0 + gc : lr * sd.sh_stride + sd.sh_col0 + (gc - 8);
    void* base = const_cast<void*>(srp ? sd.sr : sd.sh);
    if (desc->dtype == CGS_BF16) static_cast<uint16_t*>(base)[off] = f32_to_bf16_rne(v);
    else if (static_cast<float*>(base) + off != m) static_cast<float*>(base)[off] = v;
}

// ------------------------------------------------------------ chain rule
// The Gaussian's SH coefficients as the chain rule holds them across its view
// loop.  BF16 rows stay packed, two values per register, and are widened at
// each use (exact); `pin` makes the packed words opaque so the widened values
// are not kept live across the loop.  This halves the registers the rows hold
// beside the 3 NCO gradient accumulators.
template <int DT, int SHD>
struct ShRegs {
    static constexpr int N = 3 * (SHD + 1) * (SHD + 1);
    float v[N];
    __device__ void load(const SceneDesc&, int64_t, const GaussParams& gp, bool, int64_t = -1) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = gp.sh[i];
    }
    __device__ float operator[](int i) const { return v[i]; }
    __device__ void pin() {}
};

template <int SHD>
struct ShRegs<CGS_BF16, SHD> {
    static constexpr int N = 3 * (SHD + 1) * (SHD + 1);
    uint32_t w[(N + 1) / 2];
    __device__ void load(const SceneDesc& sd, int64_t g, const GaussParams&, bool vec, int64_t known = -1) {
        const uint16_t* row = static_cast<const uint16_t*>(sd.sh) + (known >= 0 ? known : (int64_t)sd.idx_sh[g]) * sd.sh_stride +
                              sd.sh_col0;
        if constexpr (N % 8 == 0) {
            if (vec) {      // host-checked: 16-byte aligned rows
                const uint4* r4 = reinterpret_cast<const uint4*>(row);
#pragma unroll
                for (int k = 0; k < N / 8; ++k) {
                    const uint4 u = r4[k];
                    w[4 * k] = u.x; w[4 * k + 1] = u.y; w[4 * k + 2] = u.z; w[4 * k + 3] = u.w;
                }
                return;
            }
        }
#pragma unroll
        for (int k = 0; k < (N + 1) / 2; ++k)
            w[k] = (uint32_t)row[2 * k] | (2 * k + 1 < N ? (uint32_t)row[2 * k + 1] << 16 : 0u);
    }
    __device__ float operator[](int i) const {
        const uint32_t x = w[i >> 1];
        return __uint_as_float((i & 1) ? (x & 0xffff0000u) : (x << 16));
    }
    __device__ void pin() {
#pragma unroll
        for (int k = 0; k < (N + 1) / 2; ++k) asm volatile("" : "+v"(w[k]));
    }
};

// fma and reciprocal in the arithmetic of the chain rule: FP32 for every
// Gaussian (the hardware reciprocal, 1 ulp), FP64 for the near-degenerate
// ones (below).
__device__ inline float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_r(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_r(double x) { return 1.0 / x; }

// The shape, projection and conic the FP32 chain rule differentiates: the
// forward's formulas with the hardware exp and reciprocals in place of the
// skeleton's exp and IEEE divisions.  The skeleton's bits decide integers in
// the forward (culling, depth keys, tile rectangles) and stay bitwise there;
// the chain rule needs the derivatives at the same point, which a few ulp do
// not move.  No cull test beyond the near plane (the same test as the
// forward's, on the same camera point): a record with a nonzero gradient was
// kept by the forward.
__device__ inline void chain_shape_of(const GaussParams& gp, GaussShape& o) {
#pragma unroll
    for (int i = 0; i < 3; ++i) o.s[i] = __expf(fminf(80.f, fmaxf(-80.f, gp.ls[i])));
    float w = gp.q[0], x = gp.q[1], y = gp.q[2], z = gp.q[3];
    const float n2 = w * w + x * x + y * y + z * z;
    if (n2 > 0.0f) {
        const float len = __builtin_sqrtf(n2);     // a normal number for any n2 > 0
        const float il = __builtin_amdgcn_rcpf(len);
        o.qlen = len;
        w *= il; x *= il; y *= il; z *= il;
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
            o.S[i][j] = o.M[i][0] * o.M[j][0] + o.M[i][1] * o.M[j][1] + o.M[i][2] * o.M[j][2];
            o.S[j][i] = o.S[i][j];
        }
}

__device__ inline bool project_chain(const ViewDesc& vd, const float* mu, const GaussShape& sh, ViewProj& p) {
    float xc, yc, zc;
    camera_point(vd, mu, xc, yc, zc);
    p.xc = xc; p.yc = yc; p.zc = zc;
    if (!(zc > kNear)) return false;
    const float iz = __builtin_amdgcn_rcpf(zc);
    const float tx = xc * iz, ty = yc * iz;
    const float txc = fminf(vd.limx, fmaxf(-vd.limx, tx));
    const float tyc = fminf(vd.limy, fmaxf(-vd.limy, ty));
    p.tx = tx; p.ty = ty; p.txc = txc; p.tyc = tyc;
    p.clx = !(tx >= -vd.limx && tx <= vd.limx);
    p.cly = !(ty >= -vd.limy && ty <= vd.limy);
    p.j00 = vd.fx * iz;
    p.j02 = -(vd.fx * txc) * iz;
    p.j11 = vd.fy * iz;
    p.j12 = -(vd.fy * tyc) * iz;
    const float* Rt = vd.Rt;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        p.T[0][j] = p.j00 * Rt[0 + j] + p.j02 * Rt[8 + j];
        p.T[1][j] = p.j11 * Rt[4 + j] + p.j12 * Rt[8 + j];
    }
    float U[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) U[a][j] = p.T[a][0] * sh.S[0][j] + p.T[a][1] * sh.S[1][j] + p.T[a][2] * sh.S[2][j];
    p.a = U[0][0] * p.T[0][0] + U[0][1] * p.T[0][1] + U[0][2] * p.T[0][2] + kBlur;
    p.c = U[1][0] * p.T[1][0] + U[1][1] * p.T[1][1] + U[1][2] * p.T[1][2] + kBlur;
    p.b = U[0][0] * p.T[1][0] + U[0][1] * p.T[1][1] + U[0][2] * p.T[1][2];
    return true;
}

// The conic with the forward's island test (FP64 when the FP32 determinant
// has lost its leading digits; those Gaussians are redone by k_chain_fp64).
__device__ inline bool conic_chain(float a, float b, float c, float& A, float& B, float& C) {
    const float det = a * c - b * b;
    if (det > 0x1p-10f * (a * c)) {
        const float id = __builtin_amdgcn_rcpf(det);
        A = c * id; B = -b * id; C = a * id;
        return false;
    }
    const double da = a, db = b, dc = c;
    const double id = 1.0 / (da * dc - db * db);
    A = (float)(dc * id); B = (float)(-db * id); C = (float)(da * id);
    return true;
}

// One view's projected-parameter gradient d = dL/d(u, v, -A/2, -B, -C/2,
// opacity, r, g, b) pulled back through the conic (A, B, C) = Sigma2D^-1,
// Sigma2D = T Sigma T^T (T = J W) and the perspective Jacobian to the camera
// point and the mean: accumulates dL/dSigma (3x3) and dL/dmean.  In `Real`
// arithmetic (the inputs -- the FP32 projection, shape and record gradient --
// are exact in either).
template <typename Real>
__device__ inline void chain_geometry(const ViewDesc& vd, const ViewProj& p, const GaussShape& sh, Real A, Real B,
                                      Real C, const float* d, Real (&dSig)[3][3], Real (&dmu)[3]) {
    // conic (A, B, C) gradient from the stored (-A/2, -B, -C/2)
    const Real dA = Real(-0.5f) * d[2], dB = -Real(d[3]), dC = Real(-0.5f) * d[4];
    // dL/dSigma2D (symmetric-matrix gradient) = -K Gk K, Gk = [[dA, dB/2], [dB/2, dC]]
    const Real hb = Real(0.5f) * dB;
    const Real m00 = A * dA + B * hb, m01 = A * hb + B * dC;
    const Real m10 = B * dA + C * hb, m11 = B * hb + C * dC;
    const Real G00 = -(m00 * A + m01 * B);
    const Real G01 = -(m00 * B + m01 * C);
    const Real G11 = -(m10 * B + m11 * C);
    // dSigma3D += T^T G T ; dT = 2 G T Sigma
    Real GT[2][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        GT[0][j] = G00 * p.T[0][j] + G01 * p.T[1][j];
        GT[1][j] = G01 * p.T[0][j] + G11 * p.T[1][j];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            dSig[i][j] = fma_r(Real(p.T[0][i]), GT[0][j], fma_r(Real(p.T[1][i]), GT[1][j], dSig[i][j]));
    Real dT[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            dT[a][j] = Real(2.f) * (GT[a][0] * sh.S[0][j] + GT[a][1] * sh.S[1][j] + GT[a][2] * sh.S[2][j]);
    // T = J W  ->  dJ = dT W^T (only the non-zero entries of J matter)
    const float* Wm = vd.Rt;   // rows at 0, 4, 8
    const Real dJ00 = dT[0][0] * Wm[0] + dT[0][1] * Wm[1] + dT[0][2] * Wm[2];
    const Real dJ02 = dT[0][0] * Wm[8] + dT[0][1] * Wm[9] + dT[0][2] * Wm[10];
    const Real dJ11 = dT[1][0] * Wm[4] + dT[1][1] * Wm[5] + dT[1][2] * Wm[6];
    const Real dJ12 = dT[1][0] * Wm[8] + dT[1][1] * Wm[9] + dT[1][2] * Wm[10];
    const Real iz = rcp_r(Real(p.zc)), iz2 = iz * iz;
    // camera-space gradient
    Real gx = Real(d[0]) * vd.fx * iz;
    Real gy = Real(d[1]) * vd.fy * iz;
    Real gz = -(Real(d[0]) * vd.fx * p.xc + Real(d[1]) * vd.fy * p.yc) * iz2;
    gz += -(dJ00 * vd.fx + dJ11 * vd.fy) * iz2;
    if (!p.clx) {   // J02 = -fx x / z^2
        gx += dJ02 * (-vd.fx * iz2);
        gz += dJ02 * (Real(2.f) * vd.fx * p.xc * iz2 * iz);
    } else {        // J02 = -fx txc / z, txc constant
        gz += dJ02 * (Real(vd.fx) * p.txc * iz2);
    }
    if (!p.cly) {
        gy += dJ12 * (-vd.fy * iz2);
        gz += dJ12 * (Real(2.f) * vd.fy * p.yc * iz2 * iz);
    } else {
        gz += dJ12 * (Real(vd.fy) * p.tyc * iz2);
    }
    // x_c = W mu + t  ->  dmu += W^T dx_c
    dmu[0] += Wm[0] * gx + Wm[4] * gy + Wm[8] * gz;
    dmu[1] += Wm[1] * gx + Wm[5] * gy + Wm[9] * gz;
    dmu[2] += Wm[2] * gx + Wm[6] * gy + Wm[10] * gz;
}

// One view's colour gradient: c = max(0, sum Y k + 1/2) with Y of the unit
// direction camera -> mean; bit ch of cm says the forward's channel ch was
// above the clamp (its value, not recomputed here).  Accumulates dL/dk into
// dk and, for SH degree >= 1, writes the direction's contribution to dL/dmean
// into gdir.
template <int DT, int SHD>
__device__ inline void chain_colour(const ViewDesc& vd, const GaussParams& gp, ShRegs<DT, SHD>& shc, const float* d,
                                    uint32_t cm, float* dk, float* gdir) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
        shc.pin();
        float ex = gp.mean[0] - vd.campos[0], ey = gp.mean[1] - vd.campos[1], ez = gp.mean[2] - vd.campos[2];
        const float il = rsqrtf(ex * ex + ey * ey + ez * ez);
        const float x = ex * il, y = ey * il, z = ez * il;
        float Y[16];
        sh_basis<SHD>(x, y, z, Y);
        float dcol[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) dcol[ch] = ((cm >> ch) & 1u) ? d[6 + ch] : 0.f;
#pragma unroll
        for (int j = 0; j < NCO; ++j)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) dk[3 * j + ch] = fmaf(Y[j], dcol[ch], dk[3 * j + ch]);
        if constexpr (SHD >= 1) {
            shc.pin();
            float e[16];
#pragma unroll
            for (int j = 0; j < NCO; ++j)
                e[j] = dcol[0] * shc[3 * j] + dcol[1] * shc[3 * j + 1] + dcol[2] * shc[3 * j + 2];
            float qx = -kY1 * e[3], qy = -kY1 * e[1], qz = kY1 * e[2];
            if constexpr (SHD >= 2) {
                qx += kY2a * y * e[4] - kY2a * z * e[7] - 2.f * kY2b * x * e[6] + 2.f * kY2c * x * e[8];
                qy += kY2a * x * e[4] - kY2a * z * e[5] - 2.f * kY2b * y * e[6] - 2.f * kY2c * y * e[8];
                qz += -kY2a * y * e[5] - kY2a * x * e[7] + 4.f * kY2b * z * e[6];
                if constexpr (SHD >= 3) {
                    const float xx = x * x, yy = y * y, zz = z * z;
                    qx += -kY3a * 6.f * x * y * e[9] + kY3b * y * z * e[10] + kY3c * 2.f * x * y * e[11]
                          - kY3d * 6.f * x * z * e[12] - kY3c * (4.f * zz - 3.f * xx - yy) * e[13]
                          + kY3e * 2.f * x * z * e[14] - kY3a * (3.f * xx - 3.f * yy) * e[15];
                    qy += -kY3a * (3.f * xx - 3.f * yy) * e[9] + kY3b * x * z * e[10]
                          - kY3c * (4.f * zz - xx - 3.f * yy) * e[11] - kY3d * 6.f * y * z * e[12]
                          + kY3c * 2.f * x * y * e[13] - kY3e * 2.f * y * z * e[14] + kY3a * 6.f * x * y * e[15];
                    qz += kY3b * x * y * e[10] - kY3c * 8.f * y * z * e[11]
                          + kY3d * (6.f * zz - 3.f * xx - 3.f * yy) * e[12] - kY3c * 8.f * x * z * e[13]
                          + kY3e * (xx - yy) * e[14];
                }
            }
            // through the normalisation dir = e / |e|
            const float dd = qx * x + qy * y + qz * z;
            gdir[0] = (qx - x * dd) * il;
            gdir[1] = (qy - y * dd) * il;
            gdir[2] = (qz - z * dd) * il;
        }
}

// Sigma = M M^T -> dM = (G + G^T) M with M = R diag(s): dL/ds and, through
// R(q) and the normalisation of q, dL/dq (stored quaternion).
template <typename Real>
__device__ inline void chain_shape(const Real (&dSig)[3][3], const GaussShape& sh, Real (&ds)[3], Real (&dq)[4]) {
    Real dR[3][3];
    ds[0] = ds[1] = ds[2] = Real(0.f);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const Real dM = (dSig[i][0] + dSig[0][i]) * sh.M[0][j] + (dSig[i][1] + dSig[1][i]) * sh.M[1][j] +
                            (dSig[i][2] + dSig[2][i]) * sh.M[2][j];
            dR[i][j] = dM * sh.s[j];
            ds[j] = fma_r(dM, Real(sh.R[i][j]), ds[j]);
        }
    const Real w = sh.qn[0], x = sh.qn[1], y = sh.qn[2], z = sh.qn[3];
    const Real two = Real(2.f);
    Real dqw = two * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
    Real dqx = two * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - two * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                      w * dR[2][1] - two * x * dR[2][2]);
    Real dqy = two * (-two * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                      z * dR[2][1] - two * y * dR[2][2]);
    Real dqz = two * (-two * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - two * z * dR[1][1] +
                      y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
    dq[0] = dq[1] = dq[2] = dq[3] = Real(0.f);
    if (sh.qlen > 0.f) {
        const Real proj = dqw * w + dqx * x + dqy * y + dqz * z;
        const Real il = rcp_r(Real(sh.qlen));
        dq[0] = (dqw - w * proj) * il;
        dq[1] = (dqx - x * proj) * il;
        dq[2] = (dqy - y * proj) * il;
        dq[3] = (dqz - z * proj) * il;
    }
}

// Writes one Gaussian's gradients: the row [dls 3, dq 4, dlogit 1, dsh 3 NCO]
// (16-byte stores when the row is a whole number of float4s), dL/dmean and,
// for per-Gaussian opacity, dL/dlogit.
template <int SHD>
__device__ inline void store_gaussian_grad(const SceneDesc& sd, float* out, int64_t g, const float* dls,
                                           const float* dq, float dlogit, const float* dk, const float* dmu) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    if constexpr ((8 + 3 * NCO) % 4 == 0) {     // row is a whole number of float4s (16-byte aligned)
        float4* o4 = reinterpret_cast<float4*>(out);
        o4[0] = make_float4(dls[0], dls[1], dls[2], dq[0]);
        o4[1] = make_float4(dq[1], dq[2], dq[3], dlogit);
#pragma unroll
        for (int i = 0; i < (3 * NCO) / 4; ++i)
            o4[2 + i] = make_float4(dk[4 * i], dk[4 * i + 1], dk[4 * i + 2], dk[4 * i + 3]);
    } else {
        out[0] = dls[0];
        out[1] = dls[1];
        out[2] = dls[2];
        out[3] = dq[0]; out[4] = dq[1]; out[5] = dq[2]; out[6] = dq[3];
        out[7] = dlogit;
#pragma unroll
        for (int i = 0; i < 3 * NCO; ++i) out[8 + i] = dk[i];
    }
    if (sd.g_means) {
        sd.g_means[3 * g + 0] = dmu[0];
        sd.g_means[3 * g + 1] = dmu[1];
        sd.g_means[3 * g + 2] = dmu[2];
    }
    if (sd.opacity_mode == 0 && sd.g_opacity) sd.g_opacity[g] = dlogit;
}

// The codebook gradient row a global row index lands in.
struct RowOut {
    float* ptr;
    int64_t stride;
    int32_t col0;
};

__device__ inline RowOut row_out(const BatchDesc* desc, int part, int64_t row, int64_t* local, int* scene) {
    int lo = 0, hi = desc->n_scenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t off = part == 0 ? desc->scenes[mid].sr_row_off : desc->scenes[mid].sh_row_off;
        if (off <= row) lo = mid; else hi = mid - 1;
    }
    const SceneDesc& sd = desc->scenes[lo];
    *scene = lo;
    if (part == 0) {
        *local = row - sd.sr_row_off;
        return RowOut{sd.g_sr, sd.g_sr_stride, sd.g_sr_col0};
    }
    *local = row - sd.sh_row_off;
    return RowOut{sd.g_sh, sd.g_sh_stride, sd.g_sh_col0};
}

// The chain rule of one Gaussian (one lane): recompute the projection of
// every view of its scene, pull dL/d(record) back to dL/dmean and to the row
// gradient row = [dls 3, dq 4, dlogit 1, dsh 3 NCO].  Returns whether the
// footprint took the FP64 conic in some view (near-degenerate, very
// elongated): such a Gaussian's chain rule is redone in FP64 by
// k_chain_fp64.  Lanes with !inb or an invalid row get zeros.
template <int DT, int SHD>
__device__ inline bool chain_gaussian(const BatchDesc* __restrict__ desc, const SceneDesc& sd, int64_t g, bool inb,
                                      const float* __restrict__ rec_grad, const uint32_t* __restrict__ rec_flag,
                                      float* row, float (&dmu)[3], int64_t known_row = -1) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    GaussParams gp;
    const bool valid = inb && (known_row >= 0 ? load_gaussian_row<DT, SHD>(sd, g, known_row, gp, desc->vec_rows != 0)
                                              : load_gaussian<DT, SHD>(sd, g, gp, desc->vec_rows != 0));
    GaussShape sh;
    float opac = 0.f;
    ShRegs<DT, SHD> shc;
    if (valid) {
        chain_shape_of(gp, sh);
        opac = __builtin_amdgcn_rcpf(1.0f + __expf(-gp.logit));
        shc.load(sd, g, gp, desc->vec_rows != 0, known_row);
    }
    dmu[0] = dmu[1] = dmu[2] = 0.f;
    float dSig[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float* dk = row + 8;
#pragma unroll
    for (int i = 0; i < 3 * NCO; ++i) dk[i] = 0.f;
    float dop = 0.f;
    // dL/d(record) of the next view is loaded while this view's math runs
    // (no load for records with a zero sum).  The record's flags -- nonzero
    // sum, and the three colour channels the forward did not clamp -- come in
    // one 16-byte load; a Gaussian's views share a line.
    float pre[9];
    uint32_t pre_cm = 0u;
    const uint32_t* flags = rec_flag + 8 * (sd.flag_wave_off + (g >> 6) * sd.vcount) + 4 * ((g >> 5) & 1);
    auto fetch_rec = [&](int vi) {
        const ViewDesc& v = desc->views[desc->view_list[sd.vfirst + vi]];
        uint4 fw = make_uint4(0u, 0u, 0u, 0u);
        if (inb) fw = *reinterpret_cast<const uint4*>(flags + 8 * vi);
        const uint32_t b = (uint32_t)g & 31u;
        pre_cm = ((fw.y >> b) & 1u) | (((fw.z >> b) & 1u) << 1) | (((fw.w >> b) & 1u) << 2);
        const float* src = rec_grad + 9 * (v.rec_off + g);
#pragma unroll
        for (int i = 0; i < 9; ++i) pre[i] = 0.f;
        if ((fw.x >> b) & 1u)
#pragma unroll
            for (int i = 0; i < 9; ++i) pre[i] = src[i];
    };
    if (sd.vcount > 0) fetch_rec(0);

    bool isl = false;
    for (int vi = 0; vi < sd.vcount; ++vi) {
        const int v = desc->view_list[sd.vfirst + vi];
        const ViewDesc& vd = desc->views[v];
        float d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = pre[i];
        const uint32_t cm = pre_cm;
        if (vi + 1 < sd.vcount) fetch_rec(vi + 1);
        bool nz = false;
#pragma unroll
        for (int i = 0; i < 9; ++i) nz |= d[i] != 0.f;
        if (!nz || !valid) continue;
        ViewProj p;
        if (!project_chain(vd, gp.mean, sh, p)) continue;
        float A, B, C;
        isl |= conic_chain(p.a, p.b, p.c, A, B, C);
        dop += d[5];
        chain_geometry<float>(vd, p, sh, A, B, C, d, dSig, dmu);
        if constexpr (SHD >= 1) {
            float gdir[3];
            chain_colour<DT, SHD>(vd, gp, shc, d, cm, dk, gdir);
            dmu[0] += gdir[0];
            dmu[1] += gdir[1];
            dmu[2] += gdir[2];
        } else {
            chain_colour<DT, SHD>(vd, gp, shc, d, cm, dk, nullptr);
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) row[i] = 0.f;
    if (valid) {
        // the shape again (bitwise the same) rather than R, M held across the loop
#pragma unroll
        for (int i = 0; i < 3; ++i) asm volatile("" : "+v"(gp.ls[i]));
#pragma unroll
        for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(gp.q[i]));
        chain_shape_of(gp, sh);
        float ds[3], dq[4];
        chain_shape<float>(dSig, sh, ds, dq);
#pragma unroll
        for (int i = 0; i < 3; ++i) row[i] = ds[i] * sh.s[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) row[3 + i] = dq[i];
        row[7] = dop * opac * (1.f - opac);
    }
    return isl;
}

// The per-Gaussian outputs beside the row: dL/dmean, dL/dlogit of a
// per-Gaussian opacity, and the island mark (a bit per Gaussian, two words
// per wavefront of the scene, plus one word that says some bit is set) or
// the SGLD update of the Gaussian's own parameters.
__device__ inline void gaussian_epilogue(const BatchDesc* __restrict__ desc, const SceneDesc& sd, int s, int64_t g,
                                         const float* dmu, float dlogit, bool isl, uint32_t* __restrict__ isl_flag) {
    if (sd.g_means) {
        sd.g_means[3 * g + 0] = dmu[0];
        sd.g_means[3 * g + 1] = dmu[1];
        sd.g_means[3 * g + 2] = dmu[2];
    }
    if (sd.opacity_mode == 0 && sd.g_opacity) sd.g_opacity[g] = dlogit;
    if (isl) {
        atomicOr(&isl_flag[2 * (sd.wave_off + (g >> 6)) + ((g >> 5) & 1)], 1u << (g & 31));
        atomicOr(&isl_flag[2 * desc->n_gauss_waves], 1u);
    } else if (desc->sgld) {
        sgld_gaussian(desc, sd, s, g, dmu, dlogit);
    }
}

// One thread per Gaussian, in Gaussian order: the chain rule, and the
// per-Gaussian row gradient written to gtheta (for the reduction by rows that
// follows).  Island Gaussians' rows are overwritten by k_chain_fp64.
template <int DT, int SHD>
__global__ __launch_bounds__(256) void k_chain(const BatchDesc* __restrict__ desc, const float* __restrict__ rec_grad,
                                               const uint32_t* __restrict__ rec_flag,
                                               float* __restrict__ gtheta, uint32_t* __restrict__ isl_flag) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    constexpr int RW = 8 + 3 * NCO;                      // the row width of the batch's SH degree
    constexpr int kHalf = 32;                            // rows staged per round
    // Per wave: half of its gradient rows at a time, written out as whole
    // lines (a lane's own 16-byte stores would touch a line per lane).
    // Staging the record gradients the same way costs 20 registers and a
    // wave per SIMD, more than it saves.
    __shared__ __align__(16) float s_stage[4][kHalf * RW];
    const int64_t wv = wave_id(4);
    if (wv >= desc->n_gauss_waves) return;
    const int s = find_scene_by_wave(desc, wv);
    const SceneDesc& sd = desc->scenes[s];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = wv - sd.wave_off;
    const int64_t g = q * kWave + lane;
    const bool inb = g < sd.n;                  // every lane stays: the staging is wave-wide
    const int nrows = (int)(sd.n - q * kWave < kWave ? sd.n - q * kWave : kWave);
    float* stg = s_stage[w];

    float row[RW], dmu[3];
    const bool isl = chain_gaussian<DT, SHD>(desc, sd, g, inb, rec_grad, rec_flag, row, dmu);
    // rows [sd.g_off + 64 q, + nrows) are contiguous: two rounds of 32
    float* rows = gtheta + (sd.g_off + q * kWave) * RW;
#pragma unroll
    for (int h = 0; h < kWave / kHalf; ++h) {
        const int nr = nrows - h * kHalf < kHalf ? nrows - h * kHalf : kHalf;
        if (nr <= 0) break;
        if (lane >= h * kHalf && lane < h * kHalf + nr) {
            float* o = stg + (lane - h * kHalf) * RW;
#pragma unroll
            for (int i = 0; i < RW; ++i) o[i] = row[i];
        }
        wave_sync();
        float* dst = rows + (int64_t)h * kHalf * RW;
        if constexpr (RW % 4 == 0) {      // 16-byte aligned rows: one float4 per lane per store
            const int n4 = nr * (RW / 4);
            const float4* s4 = reinterpret_cast<const float4*>(stg);
#pragma unroll
            for (int it = 0; it < (kHalf * RW / 4 + kWave - 1) / kWave; ++it) {
                const int t = it * kWave + lane;
                if (t < n4) reinterpret_cast<float4*>(dst)[t] = s4[t];
                asm volatile("" ::: "memory");   // one float4 in flight: no registers held for the copy
            }
        } else {
            const int n1 = nr * RW;
#pragma unroll
            for (int it = 0; it < (kHalf * RW + kWave - 1) / kWave; ++it) {
                const int t = it * kWave + lane;
                if (t < n1) dst[t] = stg[t];
                asm volatile("" ::: "memory");
            }
        }
        wave_sync();
    }
    if (inb) gaussian_epilogue(desc, sd, s, g, dmu, row[7], isl, isl_flag);
}

// Single-codebook layout: the chain rule fused with the reduction by rows.
// The Gaussians sorted by (row, Gaussian) keep each scene in its own range
// of positions (a row key never leaves its scene's rows), so wavefront
// (scene s, q) takes positions g_off + [64 q, 64 q + 64) of that order: its
// lanes hold a few runs of equal rows.  The rows are staged in LDS and lane c
// sums column c of each run in position order.  A run holding all of its
// row's Gaussians is the row's gradient, written to the codebook gradient
// (with the row's SGLD update); otherwise it is the head (starting at lane 0)
// or tail partial of the row in this wavefront, kept in rpart[2 wv] or
// rpart[2 wv + 1] for k_merge_rows.  Island Gaussians add zero here;
// k_merge_rows adds their FP64 rows.
template <int DT, int SHD>
__global__ __launch_bounds__(256) void k_chain_rows(const BatchDesc* __restrict__ desc,
                                                    const float* __restrict__ rec_grad,
                                                    const uint32_t* __restrict__ rec_flag,
                                                    const uint32_t* __restrict__ skey, const uint32_t* __restrict__ sval,
                                                    const uint32_t* __restrict__ row_range, float* __restrict__ rpart,
                                                    uint32_t* __restrict__ isl_flag) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    constexpr int RW = 8 + 3 * NCO;
    constexpr int kHalf = 32;
    __shared__ __align__(16) float s_stage[4][kHalf * RW];
    const int64_t wv = wave_id(4);
    if (wv >= desc->n_gauss_waves) return;
    const int s = find_scene_by_wave(desc, wv);
    const SceneDesc& sd = desc->scenes[s];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = wv - sd.wave_off;
    const int64_t p0 = sd.g_off + q * kWave;                  // the wavefront's first sorted position
    const int nlive = (int)(sd.n - q * kWave < kWave ? sd.n - q * kWave : kWave);
    const bool live = lane < nlive;
    const uint32_t key = live ? skey[p0 + lane] : 0xffffffffu;
    const int64_t g = live ? (int64_t)sval[p0 + lane] - sd.g_off : 0;

    float row[RW], dmu[3];
    // the row is the sort key (a valid Gaussian's index; clamped otherwise)
    const int64_t known = live ? (int64_t)key - sd.sr_row_off : 0;
    const bool isl = chain_gaussian<DT, SHD>(desc, sd, g, live, rec_grad, rec_flag, row, dmu, known);
    if (live) gaussian_epilogue(desc, sd, s, g, dmu, row[7], isl, isl_flag);

    const int64_t n_rows = desc->sr_rows_total;
    const uint64_t islm = __ballot(isl);
    float* stg = s_stage[w];
    float acc = 0.f;
    uint32_t cur = __builtin_amdgcn_readfirstlane(key);
    int seg0 = 0;
    auto flush = [&](uint32_t kr, int a, int b) {
        if ((int64_t)kr >= n_rows) return;
        const uint32_t rs = row_range[2 * (int64_t)kr], re = row_range[2 * (int64_t)kr + 1];
        const bool whole = (int64_t)rs >= p0 + a && (int64_t)re <= p0 + b;
        if (whole) {
            const uint64_t span = (b - a < 64 ? (1ull << (b - a)) - 1ull : ~0ull) << a;
            int64_t lr;
            int sc;
            const RowOut o = row_out(desc, 0, kr, &lr, &sc);
            if (lane < RW) {
                o.ptr[lr * o.stride + o.col0 + lane] = acc;
                if (desc->sgld && (islm & span) == 0ull) sgld_row(desc, sc, lr, lane, acc);
            }
        } else if (lane < RW) {
            rpart[(2 * wv + (a == 0 ? 0 : 1)) * RW + lane] = acc;
        }
    };
#pragma unroll
    for (int h = 0; h < kWave / kHalf; ++h) {
        const int r0 = h * kHalf;
        if (r0 >= nlive) break;
        const int nr = nlive - r0 < kHalf ? nlive - r0 : kHalf;
        if (lane >= r0 && lane < r0 + nr) {
            float* o = stg + (lane - r0) * RW;
#pragma unroll
            for (int i = 0; i < RW; ++i) o[i] = isl ? 0.f : row[i];
        }
        wave_sync();
        for (int rr = 0; rr < nr; ++rr) {
            const int r = r0 + rr;
            const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, r);
            if (k != cur) {
                flush(cur, seg0, r);
                cur = k;
                seg0 = r;
                acc = 0.f;
            }
            if (lane < RW) acc += stg[rr * RW + lane];
        }
        wave_sync();
    }
    flush(cur, seg0, nlive);
}

// The rows k_chain_rows left partial: a row spanning several wavefronts
// (head or tail partial of each, summed in wavefront order) or holding
// island Gaussians (their FP64 rows, written to gtheta by k_chain_fp64, added
// in position order); and the rows no Gaussian maps to (a zero gradient, and
// their SGLD update).  One wavefront per row, lanes over columns.
__global__ __launch_bounds__(256) void k_merge_rows(const BatchDesc* __restrict__ desc,
                                                    const uint32_t* __restrict__ sval,
                                                    const uint32_t* __restrict__ row_range,
                                                    const float* __restrict__ rpart, const float* __restrict__ gtheta,
                                                    const uint32_t* __restrict__ isl_flag) {
    const int lane = threadIdx.x & 63;
    const int64_t r = wave_id(4);
    if (r >= desc->sr_rows_total) return;
    const int RW = desc->row_width;
    const int64_t rs = row_range[2 * r], re = row_range[2 * r + 1];
    int64_t lr;
    int sc;
    const RowOut o = row_out(desc, 0, r, &lr, &sc);
    if (rs == re) {                                         // no Gaussian maps to the row: zero gradient
        if (lane < RW) {
            o.ptr[lr * o.stride + o.col0 + lane] = 0.f;
            if (desc->sgld) sgld_row(desc, sc, lr, lane, 0.f);
        }
        return;
    }
    // the row's positions lie in its scene's range: wavefronts of that scene
    const SceneDesc& sd = desc->scenes[sc];
    const int64_t w0 = sd.wave_off + ((rs - sd.g_off) >> 6), w1 = sd.wave_off + ((re - 1 - sd.g_off) >> 6);
    auto island = [&](uint32_t gid) -> bool {
        const SceneDesc& sd = desc->scenes[find_scene(desc, gid)];
        const int64_t g = (int64_t)gid - sd.g_off;
        return (isl_flag[2 * (sd.wave_off + (g >> 6)) + ((g >> 5) & 1)] >> (g & 31)) & 1u;
    };
    bool has_isl = false;
    if (isl_flag[2 * desc->n_gauss_waves] != 0u)
        for (int64_t pb = rs; pb < re; pb += 64)
            has_isl |= __ballot(pb + lane < re && island(sval[pb + lane])) != 0ull;
    if (w0 == w1 && !has_isl) return;                       // written whole by k_chain_rows
    float* out = o.ptr + lr * o.stride + o.col0;
    float acc = 0.f;
    if (lane < RW) {
        if (w0 == w1) {
            acc = out[lane];                                // the run's sum, islands left out
        } else {
            const bool head = ((rs - sd.g_off) & 63) == 0;    // the row starts a wavefront
            acc = rpart[(2 * w0 + (head ? 0 : 1)) * RW + lane];
            // the head partials of the later wavefronts, eight loads in
            // flight, added in wavefront order (a row of a small codebook can
            // span thousands of wavefronts)
            int64_t wq = w0 + 1;
            for (; wq + 8 <= w1 + 1; wq += 8) {
                float a[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) a[t] = rpart[2 * (wq + t) * RW + lane];
#pragma unroll
                for (int t = 0; t < 8; ++t) acc += a[t];
            }
            for (; wq <= w1; ++wq) acc += rpart[2 * wq * RW + lane];
        }
    }
    if (has_isl)
        for (int64_t pp = rs; pp < re; ++pp) {
            const uint32_t gid = sval[pp];
            if (island(gid) && lane < RW) acc += gtheta[(int64_t)gid * RW + lane];
        }
    if (lane < RW) {
        out[lane] = acc;
        if (desc->sgld) sgld_row(desc, sc, lr, lane, acc);
    }
}

// The chain rule of the Gaussians k_chain marked, in FP64 from the conic on:
// the conic is the FP64 inverse of the FP32 Sigma2D (the forward's island),
// and dL/dSigma2D = -K Gk K, dL/dSigma, dL/dmean through the Jacobian and
// dL/d(s, q) are carried in FP64.  For such a footprint the rotation's share
// of dL/dSigma2D is about 1e-3 of its largest entry, below what FP32 keeps.
// One thread per flag word; its set bits are processed in order.
template <int DT, int SHD>
__global__ __launch_bounds__(256) void k_chain_fp64(const BatchDesc* __restrict__ desc,
                                                    const float* __restrict__ rec_grad,
                                                    const uint32_t* __restrict__ rec_flag, float* __restrict__ gtheta,
                                                    const uint32_t* __restrict__ isl_flag) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= 2 * desc->n_gauss_waves) return;
    uint32_t bits = isl_flag[w];
    if (!bits) return;
    const int64_t wv = w >> 1;
    const int s = find_scene_by_wave(desc, wv);
    const SceneDesc& sd = desc->scenes[s];
    while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1;
        const int64_t g = (wv - sd.wave_off) * kWave + 32 * (w & 1) + b;
        if (g >= sd.n) break;
        GaussParams gp;
        if (!load_gaussian<DT, SHD>(sd, g, gp, desc->vec_rows != 0)) continue;
        GaussShape sh;
        gaussian_shape(gp, sh);
        const float opac = 1.0f / (1.0f + __expf(-gp.logit));
        ShRegs<DT, SHD> shc;
        shc.load(sd, g, gp, desc->vec_rows != 0);
        double dmu[3] = {0.0, 0.0, 0.0};
        double dSig[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        float dk[48];
#pragma unroll
        for (int i = 0; i < 3 * NCO; ++i) dk[i] = 0.f;
        float dop = 0.f;
        for (int vi = 0; vi < sd.vcount; ++vi) {
            const ViewDesc& vd = desc->views[desc->view_list[sd.vfirst + vi]];
            const uint4 fw = *reinterpret_cast<const uint4*>(rec_flag + 8 * (sd.flag_wave_off + (g >> 6) * sd.vcount + vi) +
                                                             4 * ((g >> 5) & 1));
            const uint32_t b = (uint32_t)g & 31u;
            if (!((fw.x >> b) & 1u)) continue;
            const uint32_t cm = ((fw.y >> b) & 1u) | (((fw.z >> b) & 1u) << 1) | (((fw.w >> b) & 1u) << 2);
            float d[9];
            const float* src = rec_grad + 9 * (vd.rec_off + g);
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = src[i];
            bool nz = false;
#pragma unroll
            for (int i = 0; i < 9; ++i) nz |= d[i] != 0.f;
            if (!nz) continue;
            ViewProj p;
            if (!project_view(vd, gp.mean, sh, p)) continue;
            double A, B, C;
            conic_of_f64(p.a, p.b, p.c, A, B, C);
            dop += d[5];
            chain_geometry<double>(vd, p, sh, A, B, C, d, dSig, dmu);
            if constexpr (SHD >= 1) {
                float gdir[3];
                chain_colour<DT, SHD>(vd, gp, shc, d, cm, dk, gdir);
                dmu[0] += gdir[0];
                dmu[1] += gdir[1];
                dmu[2] += gdir[2];
            } else {
                chain_colour<DT, SHD>(vd, gp, shc, d, cm, dk, nullptr);
            }
        }
        double ds[3], dq[4];
        chain_shape<double>(dSig, sh, ds, dq);
        const float dlogit = dop * opac * (1.f - opac);
        const float dls[3] = {(float)(ds[0] * sh.s[0]), (float)(ds[1] * sh.s[1]), (float)(ds[2] * sh.s[2])};
        const float dqf[4] = {(float)dq[0], (float)dq[1], (float)dq[2], (float)dq[3]};
        const float dmuf[3] = {(float)dmu[0], (float)dmu[1], (float)dmu[2]};
        store_gaussian_grad<SHD>(sd, gtheta + (sd.g_off + g) * desc->row_width, g, dls, dqf, dlogit, dk, dmuf);
        if (desc->sgld) sgld_gaussian(desc, sd, s, g, dmuf, dlogit);
    }
}

// ------------------------------------------------- codebook row reduction
// Sort keys for the reduction: global row = row offset of the scene + index.
__global__ __launch_bounds__(256) void k_row_keys(const BatchDesc* __restrict__ desc, int part,
                                                  uint32_t* __restrict__ key) {
    const int64_t gg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gg >= desc->n_gauss) return;
    const int s = find_scene(desc, gg);
    const SceneDesc& sd = desc->scenes[s];
    const int64_t g = gg - sd.g_off;
    // an index outside the codebook (the Gaussian is invalid, its row
    // gradient zero) is clamped into the scene's rows, so every scene keeps
    // its own range of the sorted order
    const int64_t k = part == 0 ? sd.idx_sr[g] : sd.idx_sh[g];
    const int64_t rows = part == 0 ? sd.sr_rows : sd.sh_rows;
    const int64_t kc = k < 0 ? 0 : (k >= rows ? rows - 1 : k);
    key[gg] = (uint32_t)((part == 0 ? sd.sr_row_off : sd.sh_row_off) + kc);
}

// One wavefront per chunk of kReduceChunk consecutive positions of the
// row-sorted order, lanes over columns.  The wave owns every row that starts
// inside its chunk (running past the chunk's end to finish the last one) and
// sums each row's Gaussians one position at a time, so every row is a plain
// sequential sum in sorted (row, Gaussian index) order: deterministic and
// independent of where the row sits in the batch.  A row read is one
// contiguous load of D floats across the lanes.
__global__ __launch_bounds__(256) void k_reduce_rows(const BatchDesc* __restrict__ desc, int part,
                                                     const float* __restrict__ gtheta, int64_t ld, int c0, int D,
                                                     int oshift, const uint32_t* __restrict__ skey,
                                                     const uint32_t* __restrict__ sval, int64_t n, int64_t n_rows,
                                                     const uint32_t* __restrict__ row_range) {
    const int lane = threadIdx.x & 63;
    const int64_t chunk = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t p0 = chunk * kReduceChunk;
    if (p0 >= n) return;
    const int64_t pend = p0 + kReduceChunk < n ? p0 + kReduceChunk : n;
    // first row starting at or after p0
    int64_t p;
    {
        const uint32_t r = skey[p0];
        if ((int64_t)r >= n_rows) return;
        p = (int64_t)row_range[2 * (int64_t)r] == p0 ? p0 : (int64_t)row_range[2 * (int64_t)r + 1];
    }
    while (p < pend) {
        const uint32_t r = skey[p];
        if ((int64_t)r >= n_rows) break;                    // index outside the codebook: dropped
        const int64_t e = row_range[2 * (int64_t)r + 1];
        int64_t lr;
        int sc;
        const RowOut o = row_out(desc, part, r, &lr, &sc);
        for (int cb = 0; cb < D; cb += 64) {
            const int col = cb + lane;
            const bool on = col < D;
            float acc = 0.f;
            // 64 sorted Gaussian ids per coalesced load, broadcast by readlane;
            // eight rows' loads in flight; the sum keeps position order
            for (int64_t qb = p; qb < e; qb += 64) {
                const int nq = (int)(e - qb < 64 ? e - qb : 64);
                const uint32_t ids = lane < nq ? sval[qb + lane] : 0u;
                int k = 0;
                for (; k + 8 <= nq; k += 8) {
                    float a[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const uint32_t gid = (uint32_t)__builtin_amdgcn_readlane((int)ids, k + t);
                        a[t] = on ? gtheta[(int64_t)gid * ld + c0 + col] : 0.f;
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) acc += a[t];
                }
                for (; k < nq; ++k) {
                    const uint32_t gid = (uint32_t)__builtin_amdgcn_readlane((int)ids, k);
                    acc += on ? gtheta[(int64_t)gid * ld + c0 + col] : 0.f;
                }
            }
            if (on) {
                o.ptr[lr * o.stride + o.col0 + oshift + col] = acc;
                if (desc->sgld) sgld_row(desc, sc, lr, c0 + col, acc);
            }
        }
        p = e;
    }
}

// Rows no Gaussian maps to get a zero gradient.
__global__ __launch_bounds__(256) void k_reduce_empty(const BatchDesc* __restrict__ desc, int part, int c0, int D,
                                                      int oshift, int64_t n_rows,
                                                      const uint32_t* __restrict__ row_range) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_rows * D) return;
    const int64_t row = e / D;
    const int col = (int)(e - row * D);
    if (row_range[2 * row] != row_range[2 * row + 1]) return;
    int64_t lr;
    int sc;
    const RowOut o = row_out(desc, part, row, &lr, &sc);
    o.ptr[lr * o.stride + o.col0 + oshift + col] = 0.f;
    if (desc->sgld) sgld_row(desc, sc, lr, c0 + col, 0.f);
}

// Sorted keys from a caller-provided permutation: key[i] = idx[perm[i]].
__global__ __launch_bounds__(256) void k_gather_keys(const int32_t* __restrict__ idx, const int32_t* __restrict__ perm,
                                                     int64_t n, uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t g = perm[i];
    key[i] = (uint32_t)idx[g];
    val[i] = (uint32_t)g;
}

__global__ __launch_bounds__(256) void k_copy_keys(const int32_t* __restrict__ idx, int64_t n,
                                                   uint32_t* __restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint32_t)idx[i];
}

// ---------------------------------------------------------------- L1 loss
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ img, const float* __restrict__ tgt, int64_t n,
                                            float inv_n, float* __restrict__ grad, float* __restrict__ part) {
    __shared__ float s[256];
    float acc = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // 16-byte loads and stores over the aligned bulk, single values after it
    const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                       reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    for (int64_t q = t0; q < n4; q += stride) {
        const float4 a = reinterpret_cast<const float4*>(img)[q], b = reinterpret_cast<const float4*>(tgt)[q];
        const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
        acc += fabsf(d0); acc += fabsf(d1); acc += fabsf(d2); acc += fabsf(d3);
        reinterpret_cast<float4*>(grad)[q] =
            make_float4(d0 > 0.f ? inv_n : (d0 < 0.f ? -inv_n : 0.f), d1 > 0.f ? inv_n : (d1 < 0.f ? -inv_n : 0.f),
                        d2 > 0.f ? inv_n : (d2 < 0.f ? -inv_n : 0.f), d3 > 0.f ? inv_n : (d3 < 0.f ? -inv_n : 0.f));
    }
    for (int64_t i = 4 * n4 + t0; i < n; i += stride) {
        const float d = img[i] - tgt[i];
        acc += fabsf(d);
        grad[i] = d > 0.f ? inv_n : (d < 0.f ? -inv_n : 0.f);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_l1_final(const float* __restrict__ part, int nb, int64_t n,
                                                  float* __restrict__ loss) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = n > 0 ? (float)(s[0] / (double)n) : 0.f;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_blend_bwd(const BatchDesc* d_desc, int64_t n_tiles, int wpb, bool persist, const uint32_t* ranges,
                            const uint32_t* inst_rec, const float4* rec, const uint8_t* qbits, const uint32_t* dk,
                            const uint32_t* eo,
                            const float* grad_image, const float* T_final, const int32_t* n_last, float* ginst,
                            uint2* cut, DevCounters* cnt, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (persist) {
        int64_t nb = resident_blocks(reinterpret_cast<const void*>(&k_blend_bwd<1, true>), 64);
        if (nb <= 0) return hipErrorInvalidValue;
        if (nb > n_tiles) nb = n_tiles;
        hipLaunchKernelGGL((k_blend_bwd<1, true>), dim3((unsigned)nb), dim3(64), 0, st, d_desc, ranges, inst_rec, rec,
                           qbits, dk, eo, grad_image, T_final, n_last, ginst, cut, cnt);
    } else if (wpb == 1) {
        hipLaunchKernelGGL((k_blend_bwd<1, false>), dim3((unsigned)n_tiles), dim3(64), 0, st, d_desc, ranges, inst_rec,
                           rec, qbits, dk, eo, grad_image, T_final, n_last, ginst, cut, cnt);
    } else if (wpb == 2) {
        hipLaunchKernelGGL((k_blend_bwd<2, false>), dim3((unsigned)((n_tiles + 1) / 2)), dim3(128), 0, st, d_desc,
                           ranges, inst_rec, rec, qbits, dk, eo, grad_image, T_final, n_last, ginst, cut, cnt);
    } else {
        hipLaunchKernelGGL((k_blend_bwd<4, false>), dim3((unsigned)((n_tiles + 3) / 4)), dim3(256), 0, st, d_desc,
                           ranges, inst_rec, rec, qbits, dk, eo, grad_image, T_final, n_last, ginst, cut, cnt);
    }
    return hipGetLastError();
}

hipError_t launch_slot_sum(const BatchDesc* d_desc, int64_t n_rec_waves, const float* ginst, const uint32_t* eo,
                           const uint32_t* nt, const uint2* tr, const uint32_t* prect, const uint32_t* dk,
                           const uint2* cut, const DevCounters* cnt, float* rec_grad, uint32_t* rec_flag,
                           uint32_t* isl_flag, int64_t n_gauss_waves, hipStream_t st) {
    const int64_t n_isl = 2 * n_gauss_waves + 1;       // zeroed here for the chain rule
    if (n_rec_waves <= 0) return fill_u32(isl_flag, 0u, (size_t)n_isl, st);
    hipLaunchKernelGGL(k_slot_sum, dim3((unsigned)((n_rec_waves + 3) / 4)), dim3(256), 0, st, d_desc, ginst, eo,
                       nt, tr, prect, dk, cut, cnt, rec_grad, rec_flag, isl_flag, n_isl);
    return hipGetLastError();
}

// The chain rule in Gaussian order (rows to gtheta), or fused with the
// reduction by rows when skey is given (rows sorted by the single codebook's
// index; partials to rpart), then the FP64 redo of island Gaussians.
hipError_t launch_chain(const BatchDesc* d_desc, int dtype, int shd, int64_t n_gauss_waves,
                        const float* rec_grad, const uint32_t* rec_flag, float* gtheta, uint32_t* isl_flag,
                        const uint32_t* skey, const uint32_t* sval, const uint32_t* row_range, float* rpart,
                        hipStream_t st) {
    if (n_gauss_waves <= 0) return hipGetLastError();
    // isl_flag: zeroed by the record-gradient sums just before
    dim3 grid((unsigned)((n_gauss_waves + 3) / 4)), blk(256);
    dim3 grid64((unsigned)((2 * n_gauss_waves + 255) / 256));
#define CGS_CH(DT, SHD)                                                                                     \
    do {                                                                                                    \
        if (skey)                                                                                           \
            hipLaunchKernelGGL((k_chain_rows<DT, SHD>), grid, blk, 0, st, d_desc, rec_grad, rec_flag, skey,  \
                               sval, row_range, rpart, isl_flag);                                           \
        else                                                                                                \
            hipLaunchKernelGGL((k_chain<DT, SHD>), grid, blk, 0, st, d_desc, rec_grad, rec_flag, gtheta, isl_flag); \
        hipLaunchKernelGGL((k_chain_fp64<DT, SHD>), grid64, blk, 0, st, d_desc, rec_grad, rec_flag, gtheta,      \
                           isl_flag);                                                                       \
    } while (0)
    if (dtype == CGS_F32) {
        switch (shd) { case 0: CGS_CH(CGS_F32, 0); break; case 1: CGS_CH(CGS_F32, 1); break;
                       case 2: CGS_CH(CGS_F32, 2); break; default: CGS_CH(CGS_F32, 3); break; }
    } else {
        switch (shd) { case 0: CGS_CH(CGS_BF16, 0); break; case 1: CGS_CH(CGS_BF16, 1); break;
                       case 2: CGS_CH(CGS_BF16, 2); break; default: CGS_CH(CGS_BF16, 3); break; }
    }
#undef CGS_CH
    return hipGetLastError();
}

hipError_t launch_merge_rows(const BatchDesc* d_desc, int64_t n_rows, const uint32_t* sval, const uint32_t* row_range,
                             const float* rpart, const float* gtheta, const uint32_t* isl_flag, hipStream_t st) {
    if (n_rows > 0)
        hipLaunchKernelGGL(k_merge_rows, dim3((unsigned)((n_rows + 3) / 4)), dim3(256), 0, st, d_desc, sval,
                           row_range, rpart, gtheta, isl_flag);
    return hipGetLastError();
}

hipError_t launch_row_keys(const BatchDesc* d_desc, int part, int64_t n_gauss, uint32_t* key, hipStream_t st) {
    if (n_gauss <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_keys, dim3((unsigned)((n_gauss + 255) / 256)), dim3(256), 0, st, d_desc, part, key);
    return hipGetLastError();
}

hipError_t launch_reduce(const BatchDesc* d_desc, int part, const float* gtheta, int64_t ld, int c0, int D,
                         int oshift, const uint32_t* skey, const uint32_t* sval, int64_t n, int64_t n_rows,
                         const uint32_t* row_range, hipStream_t st) {
    const int64_t chunks = (n + kReduceChunk - 1) / kReduceChunk;
    if (chunks > 0)
        hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)((chunks + 3) / 4)), dim3(256), 0, st, d_desc, part, gtheta,
                           ld, c0, D, oshift, skey, sval, n, n_rows, row_range);
    if (n_rows * D > 0)
        hipLaunchKernelGGL(k_reduce_empty, dim3((unsigned)((n_rows * D + 255) / 256)), dim3(256), 0, st, d_desc, part,
                           c0, D, oshift, n_rows, row_range);
    return hipGetLastError();
}

hipError_t launch_gather_keys(const int32_t* idx, const int32_t* perm, int64_t n, uint32_t* key, uint32_t* val,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, idx, perm, n, key, val);
    return hipGetLastError();
}

hipError_t launch_copy_keys(const int32_t* idx, int64_t n, uint32_t* key, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, idx, n, key);
    return hipGetLastError();
}

hipError_t launch_l1(const float* img, const float* tgt, int64_t n, float* grad, float* loss, float* part,
                     int nb, hipStream_t st) {
    const float inv = n > 0 ? (float)(1.0 / (double)n) : 0.f;
    if (n > 0) hipLaunchKernelGGL(k_l1, dim3(nb), dim3(256), 0, st, img, tgt, n, inv, grad, part);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(256), 0, st, part, n > 0 ? nb : 0, n, loss);
    return hipGetLastError();
}

}  // namespace cgs
