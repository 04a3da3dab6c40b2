// Forward render: codebook gather + projection + SH colour (one thread per
// Gaussian, looping over the views of its scene so the gather and the
// view-independent activations are done once per batch), instance emission,
// and the front-to-back blend (paper Sec. 2.1, Eq. 1-3).
#include <algorithm>

#include "cgs_internal.h"
#include "render_common.h"
#include "wave_scan.h"

namespace cgs {

// ---------------------------------------------------------------- preprocess
template <int DT, int SHD>
__global__ __launch_bounds__(256) void k_preprocess(const BatchDesc* __restrict__ desc,
                                                    float4* __restrict__ rec, uint32_t* __restrict__ depth_key,
                                                    uint2* __restrict__ tile_rect, uint32_t* __restrict__ ntiles,
                                                    uint32_t* __restrict__ prect, uint32_t* __restrict__ chunk_tot,
                                                    uint32_t* __restrict__ krange, uint32_t* __restrict__ rec_flag,
                                                    ZeroSpans zero) {
    constexpr int NCO = (SHD + 1) * (SHD + 1);
    {   // the counters the sorts and scans of the binning start from
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)zero.n[s]; i += stride)
                zero.p[s][i] = 0u;
    }
    const int64_t wv = wave_id(4);
    if (wv >= desc->n_gauss_waves) return;
    const SceneDesc& sd = desc->scenes[find_scene_by_wave(desc, wv)];
    const int lane = threadIdx.x & 63;
    const int64_t q = wv - sd.wave_off;            // the wave's 64-Gaussian chunk of its scene
    const int64_t g = q * kWave + lane;
    const bool inb = g < sd.n;                     // lanes past the scene's end write nothing
    const int64_t nvalid = sd.n - q * kWave < kWave ? sd.n - q * kWave : kWave;   // the wave's records per view
    __shared__ float4 s_rec[4][kRecF4 * kWave];
    const int w = (int)(threadIdx.x >> 6);

    GaussParams gp;
    const bool valid = inb && load_gaussian<DT, SHD>(sd, g, gp, desc->vec_rows != 0);
    GaussShape sh;
    if (valid) gaussian_shape(gp, sh);
    const float opac = valid ? 1.0f / (1.0f + __expf(-gp.logit)) : 0.0f;

    for (int vi = 0; vi < sd.vcount; ++vi) {
        const int v = desc->view_list[sd.vfirst + vi];
        const ViewDesc& vd = desc->views[v];
        const int64_t r = vd.rec_off + g;
        ViewProj vp;
        const bool keep = valid && project_view(vd, gp.mean, sh, vp);
        // The records of this chunk own one contiguous range of backward
        // gradient slots: the chunk's total goes to chunk_tot (scanned into
        // the chunk's base later) and each record keeps its offset within
        // the chunk in the spare word of its record.
        const uint32_t nt = keep ? (uint32_t)((vp.tx1 - vp.tx0) * (vp.ty1 - vp.ty0)) : 0u;
        const uint32_t incl = wave_incl_sum_u32(nt, lane);
        if (lane == 63) chunk_tot[vd.rec_wave_off + q] = incl;
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = make_float4(0.f, 0.f, 0.f, __uint_as_float(incl - nt));
        if (inb && !keep) {
            depth_key[r] = kCulledKey;
            if (desc->pack_rect) {
                prect[r] = 0u;      // the tile count follows from the packed rectangle
            } else {
                tile_rect[r] = make_uint2(0u, 0u);
                ntiles[r] = 0u;
            }
        } else if (inb) {
            float A, B, C;
            conic_of(vp.a, vp.b, vp.c, A, B, C);
            float col[3];
            sh_colour<SHD>(vd, gp, col, nullptr);
            depth_key[r] = __float_as_uint(vp.zc);
            const uint32_t rlo = (uint32_t)vp.tx0 | ((uint32_t)vp.ty0 << 16);
            const uint32_t rhi = (uint32_t)vp.tx1 | ((uint32_t)vp.ty1 << 16);
            if (desc->pack_rect) {
                prect[r] = (uint32_t)vp.tx0 | ((uint32_t)vp.ty0 << 8) | ((uint32_t)vp.tx1 << 16) |
                           ((uint32_t)vp.ty1 << 24);
            } else {
                tile_rect[r] = make_uint2(rlo, rhi);
                ntiles[r] = nt;
            }
            r0 = make_float4(vp.u, vp.v, (-0.5f * kLog2e) * A, -kLog2e * B);
            r1 = make_float4((-0.5f * kLog2e) * C, opac, col[0], col[1]);
            r2 = make_float4(col[2], __uint_as_float(rlo), __uint_as_float(rhi), __uint_as_float(incl - nt));
        }
        // the wave's share of the depth-key range the depth sort needs:
        // max of ~key and of key over its kept records
        {
            const uint32_t kk = __float_as_uint(vp.zc);
            const bool kept = inb && keep;
            const uint32_t nlo = wave_max_u32(kept ? ~kk : 0u), hi = wave_max_u32(kept ? kk : 0u);
            if (lane == 0) {
                krange[2 * (vd.rec_wave_off + q)] = nlo;
                krange[2 * (vd.rec_wave_off + q) + 1] = hi;
            }
        }
        // Which colour channels the forward left above its clamp at zero
        // (dL/d(SH) passes through those only): a bit per record and channel,
        // two words each per wavefront, beside the words the backward sets
        // for records with a nonzero gradient -- words 8 f + 4 h + (1, 2, 3)
        // for wavefront f of the scene's Gaussian-major order and half h.
        {
            const uint64_t m0 = __ballot(r1.z > 0.f), m1 = __ballot(r1.w > 0.f), m2 = __ballot(r2.x > 0.f);
            if (lane < 6) {
                const int h = lane >= 3 ? 1 : 0, ch = lane - 3 * h;
                const uint64_t m = ch == 0 ? m0 : (ch == 1 ? m1 : m2);
                rec_flag[8 * (sd.flag_wave_off + q * sd.vcount + vi) + 4 * h + 1 + ch] = (uint32_t)(m >> (32 * h));
            }
        }
        // The wave's records are one contiguous 3 KB block: staged in LDS and
        // written 1 KB per store instruction (whole lines but at the ends).
        s_rec[w][kRecF4 * lane + 0] = r0;
        s_rec[w][kRecF4 * lane + 1] = r1;
        s_rec[w][kRecF4 * lane + 2] = r2;
        wave_sync();
        float4* dst = rec + kRecF4 * (vd.rec_off + q * kWave);
#pragma unroll
        for (int t = 0; t < kRecF4; ++t)
            if (t * kWave + lane < kRecF4 * nvalid) dst[t * kWave + lane] = s_rec[w][t * kWave + lane];
        wave_sync();
        (void)NCO;
    }
}

// ------------------------------------------------------------ capacity check
__global__ void k_capacity(DevCounters* cnt, int64_t capacity, int64_t* d_info) {
    unsigned long long m = cnt->n_inst;
    bool ok = (int64_t)m <= capacity;
    cnt->n_inst_ok = ok ? m : 0ull;
    cnt->done_fwd = 0ull;
    cnt->done_bwd = 0ull;
    for (int x = 0; x < kQueues; ++x) {
        cnt->q_fwd[x * kQueueStride] = 0ull;
        cnt->q_bwd[x * kQueueStride] = 0ull;
    }
    if (d_info) {
        d_info[0] = ok ? CGS_OK : CGS_ECAPACITY;
        d_info[1] = (int64_t)m;
    }
}

// ------------------------------------------------------------------ emission
// Wave-cooperative emission: a wavefront owns 64 consecutive records of the
// depth order; their instances occupy one contiguous range of the instance
// array, which the 64 lanes write in order, 64 instances at a time (each
// record with tiles marks the lane of its first instance in the chunk, and
// an inclusive max-scan of the marks over the wave gives every instance its
// record, carried into the next chunk), so writes are
// coalesced and a record with many tiles does not stall its wave.  Instance
// (record, tile) keys are the view's tile offset + the row-major tile index;
// tiles of a record follow row-major order.  KT: the key's storage type
// (16 bits when the batch has at most 65536 tiles).
template <typename KT>
__global__ __launch_bounds__(256) void k_emit(const BatchDesc* __restrict__ desc, const uint32_t* __restrict__ sorted_rec,
                                              const uint32_t* __restrict__ offs, const uint2* __restrict__ rect_d,
                                              const uint32_t* __restrict__ cnt_d, const DevCounters* __restrict__ cnt,
                                              KT* __restrict__ inst_key, uint32_t* __restrict__ inst_val) {
    __shared__ uint32_t s_rel[4][64], s_w[4][64], s_base[4][64], s_tx[4][64], s_r[4][64], s_mark[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j0 = ((int64_t)blockIdx.x * 4 + w) * 64;
    if (j0 >= desc->n_rec) return;
    const int64_t j = j0 + lane;
    const bool valid = j < desc->n_rec;
    // every load this wave needs is issued at once (lanes past the end read
    // the wave's first record); lane 0's offset is the wave's base
    const int64_t jc = valid ? j : j0;
    const bool emit = cnt->n_inst_ok != 0ull;
    const uint2 tr = rect_d[jc];
    const uint32_t oj = offs[jc];
    const uint32_t r = sorted_rec[jc];
    const uint32_t c = valid ? cnt_d[jc] : 0u;
    const uint32_t o0 = __builtin_amdgcn_readfirstlane(oj);
    const uint32_t rel = valid ? oj - o0 : 0u;
    uint32_t endrel = valid ? rel + c : 0u;
    endrel = wave_max_u32(endrel);
    if (!emit) return;
    // the record's view: views hold consecutive record ranges, read with
    // scalar loads (no per-lane search through memory)
    uint32_t tx = (uint32_t)desc->views[0].tiles_x, toff = (uint32_t)desc->views[0].tile_off;
    for (int v = 1; v < desc->n_views; ++v) {
        const ViewDesc& vd = desc->views[v];
        if ((int64_t)r >= vd.rec_off) { tx = (uint32_t)vd.tiles_x; toff = (uint32_t)vd.tile_off; }
    }
    if (valid && c > 0) {
        const uint32_t x0 = tr.x & 0xffffu, y0 = tr.x >> 16, x1 = tr.y & 0xffffu;
        s_w[w][lane] = x1 - x0;
        s_tx[w][lane] = tx;
        s_base[w][lane] = toff + y0 * tx + x0;
        s_r[w][lane] = r;
    }
    s_rel[w][lane] = valid ? rel : endrel;
    wave_sync();
    uint32_t carry = 0u;     // 1 + the lane of the record owning the last instance of the previous chunk
    for (uint32_t c0 = 0; c0 < endrel; c0 += 64) {
        s_mark[w][lane] = 0u;
        wave_sync();
        if (valid && c > 0 && rel >= c0 && rel < c0 + 64u) s_mark[w][rel - c0] = (uint32_t)lane + 1u;
        wave_sync();
        // the last record of the wave whose range starts at or before i
        uint32_t m = wave_incl_max_u32(s_mark[w][lane], lane);
        m = m > carry ? m : carry;
        carry = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
        const uint32_t i = c0 + (uint32_t)lane;
        if (i < endrel) {
            const int lo = (int)m - 1;
            const uint32_t local = i - s_rel[w][lo];
            const uint32_t wq = s_w[w][lo];
            uint32_t row = (uint32_t)((float)local * __builtin_amdgcn_rcpf((float)wq));
            if (row * wq > local) --row;
            if ((row + 1) * wq <= local) ++row;
            inst_key[o0 + i] = (KT)(s_base[w][lo] + row * s_tx[w][lo] + (local - row * wq));
            inst_val[o0 + i] = s_r[w][lo];
        }
        wave_sync();
    }
}

// Forward of the standalone binning call: instance keys from caller arrays.
__global__ __launch_bounds__(256) void k_emit_plain(const uint16_t* __restrict__ trect, const int32_t* __restrict__ view_of,
                                                    const uint32_t* __restrict__ sorted_rec, const uint32_t* __restrict__ offs,
                                                    int64_t n, int32_t tiles_x, int32_t tiles_y,
                                                    const DevCounters* __restrict__ cnt, uint32_t* __restrict__ inst_key,
                                                    uint32_t* __restrict__ inst_val) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (cnt->n_inst_ok == 0ull) return;
    const uint32_t r = sorted_rec[j];
    const uint32_t x0 = trect[4 * r], y0 = trect[4 * r + 1], x1 = trect[4 * r + 2], y1 = trect[4 * r + 3];
    if (x1 <= x0 || y1 <= y0) return;
    const uint32_t vw = view_of ? (uint32_t)view_of[r] : 0u;
    uint32_t o = offs[j];
    for (uint32_t ty = y0; ty < y1; ++ty)
        for (uint32_t tx = x0; tx < x1; ++tx) {
            inst_key[o] = (vw * (uint32_t)tiles_y + ty) * (uint32_t)tiles_x + tx;
            inst_val[o] = r;
            ++o;
        }
}

__global__ __launch_bounds__(256) void k_plain_counts(const uint16_t* __restrict__ trect, int64_t n,
                                                      uint32_t* __restrict__ ntiles) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t x0 = trect[4 * i], y0 = trect[4 * i + 1], x1 = trect[4 * i + 2], y1 = trect[4 * i + 3];
    ntiles[i] = (x1 > x0 && y1 > y0) ? (x1 - x0) * (y1 - y0) : 0u;
}

__global__ __launch_bounds__(256) void k_plain_keys(const uint32_t* __restrict__ sorted_tile,
                                                    const uint32_t* __restrict__ sorted_gid,
                                                    const uint32_t* __restrict__ depth_key,
                                                    const DevCounters* __restrict__ cnt, int64_t cap,
                                                    uint64_t* __restrict__ out_key, uint32_t* __restrict__ out_gid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t m = (int64_t)cnt->n_inst_ok;
    if (m > cap) m = cap;
    if (i >= m) return;
    const uint32_t gid = sorted_gid[i];
    if (out_key) out_key[i] = ((uint64_t)sorted_tile[i] << 32) | (uint64_t)depth_key[gid];
    out_gid[i] = gid;
}

// ------------------------------------------------------------ forward blend
// One wavefront per 16x16 tile.  Lane l shades pixel (l & 7, l >> 3) of each
// of the four 8x8 quadrants k (k & 1 right, k >> 1 lower).  The tile's sorted
// records are read 64 at a time (one per lane); each lane marks the quadrants
// its record can reach with alpha >= 1/255, records reaching none are
// dropped, the rest are packed in order into LDS (ballot prefix) and read
// back as wave-uniform broadcasts; a quadrant the record cannot reach is
// skipped by the whole wave.  List positions are kept, so n_last is unchanged.
// The quadrant mask of each list position is also stored for the backward
// (qbits, one byte per position, written up to where every pixel of the tile
// has terminated), or 0 when no pixel of the tile blended the record: the
// backward then skips it without re-deriving alpha.
//
// PERSIST: the grid is resident and each wavefront takes tiles from the
// forward's tile queue until it runs dry (same per-tile work and results).
template <int WPB, bool STATS, bool PERSIST>
__global__ __launch_bounds__(WPB * 64) void k_blend_fwd(const BatchDesc* __restrict__ desc,
                                                         const uint32_t* __restrict__ ranges,
                                                         const uint32_t* __restrict__ inst_rec,
                                                         const float4* __restrict__ rec,
                                                         uint8_t* __restrict__ qbits,
                                                         float* __restrict__ image, float* __restrict__ T_final,
                                                         int32_t* __restrict__ n_last, int32_t* __restrict__ n_blend,
                                                         DevCounters* __restrict__ cnt) {
    __shared__ float4 s_g[WPB][64];
    __shared__ float4 s_c[WPB][64];
    __shared__ float s_b[WPB][64];
    __shared__ uint32_t s_p[WPB][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t fetched = 0u;
    if constexpr (PERSIST) fetched = fetch_pos(cnt->q_fwd, lane);
    for (int it = 0;; ++it) {
        int64_t tile;
        if constexpr (PERSIST) {
            tile = tile_at(desc, fetched);
            if (tile < desc->n_tiles) fetched = fetch_pos(cnt->q_fwd, lane);   // the next one, waited for at the top
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
        const float bx0 = (float)x0, by0 = (float)y0;
        const float bxm = (float)min(x0 + kTile - 1, vd.W - 1), bym = (float)min(y0 + kTile - 1, vd.H - 1);

        // T > 0 while the pixel is live; a finished (or outside) pixel keeps -T,
        // so a dead lane takes the termination branch and changes nothing
        float T[4], C0[4], C1[4], C2[4], fpx[4], fpy[4];
        uint32_t last[4], nb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int px = x0 + 8 * (k & 1) + (lane & 7), py = y0 + 8 * (k >> 1) + (lane >> 3);
            T[k] = (px < vd.W && py < vd.H) ? 1.f : -1.f;
            C0[k] = C1[k] = C2[k] = 0.f; last[k] = 0; nb[k] = 0;
            fpx[k] = (float)px;
            fpy[k] = (float)py;
        }
        const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
        for (uint32_t b = start; b < end; b += 64) {
            if (__ballot((T[0] > 0.f) | (T[1] > 0.f) | (T[2] > 0.f) | (T[3] > 0.f)) == 0ull) break;
            const uint32_t idx = b + lane;
            uint32_t qm = 0u;
            float4 g, c;
            float bl = 0.f;
            if (idx < end) {
                const int64_t r = inst_rec[idx];
                g = rec[kRecF4 * r + 0];
                c = rec[kRecF4 * r + 1];
                bl = rec[kRecF4 * r + 2].x;
                qm = quadrant_mask(g, c, bx0, by0, bxm, bym);
            }
            const uint64_t km = __ballot(qm != 0u);
            const uint32_t mine = popc_below(km);
            if (qm != 0u) {
                s_g[w][mine] = g;
                s_c[w][mine] = c;
                s_b[w][mine] = bl;
                s_p[w][mine] = ((idx - start + 1u) << 4) | qm;
            }
            wave_sync();
            const int cnt = (int)__popcll(km);
            uint32_t hit_lo = 0u, hit_hi = 0u;     // staged records this lane blended (bit j)
            uint32_t qlive = 0u;
            for (int j = 0; j < cnt; ++j) {
                // quadrants with a live pixel (wave-uniform), once per staged
                // batch: a quadrant whose pixels all finish within the batch
                // is still evaluated for its later records, and its finished
                // lanes take the termination branch, which changes nothing
                // (checking before every record cost the forward 0.13 ms)
                if (j == 0) {
                    qlive = 0u;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (__ballot(T[k] > 0.f) != 0ull) qlive |= 1u << k;
                    if (qlive == 0u) break;
                }
                const float4 gg = s_g[w][j];
                const float4 cc = s_c[w][j];
                const float bb = s_b[w][j];
                const uint32_t pq = __builtin_amdgcn_readfirstlane(s_p[w][j]);
                const uint32_t pos = pq >> 4;
                const uint32_t act = pq & qlive;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (!((act >> k) & 1u)) continue;          // wave-uniform quadrant skip
                    const float dx = fpx[k] - gg.x;
                    const float dy = fpy[k] - gg.y;
                    float G;
                    bool pcl;
                    const float alpha = blend_alpha(dx, dy, gg, cc, G, pcl);
                    if (alpha < kMinAlpha) continue;
                    const float Tn = T[k] * (1.f - alpha);
                    if (Tn < kMinT) {      // finished here (or already): keep -T
                        T[k] = -fabsf(T[k]);
                        continue;
                    }
                    const float wgt = alpha * T[k];
                    C0[k] = fmaf(wgt, cc.z, C0[k]);
                    C1[k] = fmaf(wgt, cc.w, C1[k]);
                    C2[k] = fmaf(wgt, bb, C2[k]);
                    T[k] = Tn;
                    last[k] = pos;
                    if (j < 32) hit_lo |= 1u << j;     // this lane blended staged record j
                    else hit_hi |= 1u << (j - 32);
                    if constexpr (STATS) ++nb[k];
                }
            }
            hit_lo = wave_or_u32(hit_lo);
            hit_hi = wave_or_u32(hit_hi);
            const uint32_t blended = mine < 32 ? (hit_lo >> mine) & 1u : (hit_hi >> (mine - 32)) & 1u;
            if (idx < end) qbits[idx] = (qm != 0u && blended) ? (uint8_t)qm : (uint8_t)0;
            wave_sync();
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int px = x0 + 8 * (k & 1) + (lane & 7), py = y0 + 8 * (k >> 1) + (lane >> 3);
            if (px < vd.W && py < vd.H) {
                const int64_t p = vd.pix_off + (int64_t)py * vd.W + px;
                const float Tk = fabsf(T[k]);
                image[3 * p + 0] = C0[k] + Tk * vd.bg[0];
                image[3 * p + 1] = C1[k] + Tk * vd.bg[1];
                image[3 * p + 2] = C2[k] + Tk * vd.bg[2];
                T_final[p] = Tk;
                n_last[p] = (int32_t)last[k];
                if constexpr (STATS) n_blend[p] = (int32_t)nb[k];
            }
        }
    }
    if constexpr (PERSIST) retire_wave(cnt->q_fwd, &cnt->done_fwd, (unsigned long long)gridDim.x * WPB, lane);
}

// ------------------------------------------------------------------ launchers
hipError_t launch_preprocess(const BatchDesc* d_desc, int dtype, int shd, int64_t n_gauss_waves, float4* rec,
                             uint32_t* dk, uint2* tr, uint32_t* nt, uint32_t* prect, uint32_t* chunk_tot,
                             uint32_t* krange, uint32_t* rec_flag, const ZeroSpans& zero, hipStream_t st) {
    if (n_gauss_waves <= 0) {       // no preprocess launch: zero the spans by fills
        for (int s = 0; s < 4; ++s) {
            const hipError_t e = fill_u32(zero.p[s], 0u, zero.n[s], st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    dim3 grid((unsigned)((n_gauss_waves + 3) / 4)), blk(256);
#define CGS_PRE(DT, SHD) hipLaunchKernelGGL((k_preprocess<DT, SHD>), grid, blk, 0, st, d_desc, rec, dk, tr, nt, prect, chunk_tot, krange, rec_flag, zero)
    if (dtype == CGS_F32) {
        switch (shd) { case 0: CGS_PRE(CGS_F32, 0); break; case 1: CGS_PRE(CGS_F32, 1); break;
                       case 2: CGS_PRE(CGS_F32, 2); break; default: CGS_PRE(CGS_F32, 3); break; }
    } else {
        switch (shd) { case 0: CGS_PRE(CGS_BF16, 0); break; case 1: CGS_PRE(CGS_BF16, 1); break;
                       case 2: CGS_PRE(CGS_BF16, 2); break; default: CGS_PRE(CGS_BF16, 3); break; }
    }
#undef CGS_PRE
    return hipGetLastError();
}

hipError_t launch_capacity(DevCounters* cnt, int64_t capacity, int64_t* d_info, hipStream_t st) {
    hipLaunchKernelGGL(k_capacity, dim3(1), dim3(1), 0, st, cnt, capacity, d_info);
    return hipGetLastError();
}

hipError_t launch_emit(const BatchDesc* d_desc, int64_t n_rec, const uint32_t* sorted_rec, const uint32_t* offs,
                       const uint2* rect_d, const uint32_t* cnt_d, const DevCounters* cnt, void* ik, bool key16,
                       uint32_t* iv, hipStream_t st) {
    if (n_rec <= 0) return hipSuccess;
    const int64_t waves = (n_rec + 63) / 64;
    if (key16)
        hipLaunchKernelGGL(k_emit<uint16_t>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, d_desc, sorted_rec,
                           offs, rect_d, cnt_d, cnt, static_cast<uint16_t*>(ik), iv);
    else
        hipLaunchKernelGGL(k_emit<uint32_t>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, d_desc, sorted_rec,
                           offs, rect_d, cnt_d, cnt, static_cast<uint32_t*>(ik), iv);
    return hipGetLastError();
}

hipError_t launch_plain_counts(const uint16_t* trect, int64_t n, uint32_t* nt, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plain_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, trect, n, nt);
    return hipGetLastError();
}

hipError_t launch_emit_plain(const uint16_t* trect, const int32_t* view_of, const uint32_t* sorted_rec,
                             const uint32_t* offs, int64_t n, int32_t tiles_x, int32_t tiles_y,
                             const DevCounters* cnt, uint32_t* ik, uint32_t* iv, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit_plain, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, trect, view_of, sorted_rec,
                       offs, n, tiles_x, tiles_y, cnt, ik, iv);
    return hipGetLastError();
}

hipError_t launch_plain_keys(const uint32_t* stile, const uint32_t* sgid, const uint32_t* dkey, const DevCounters* cnt,
                             int64_t cap, uint64_t* out_key, uint32_t* out_gid, hipStream_t st) {
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plain_keys, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, st, stile, sgid, dkey, cnt, cap,
                       out_key, out_gid);
    return hipGetLastError();
}


hipError_t launch_blend_fwd(const BatchDesc* d_desc, int64_t n_tiles, int wpb, bool persist, const uint32_t* ranges,
                            const uint32_t* inst_rec, const float4* rec, uint8_t* qbits,
                            float* image, float* T_final, int32_t* n_last, int32_t* n_blend, DevCounters* cnt,
                            hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (persist) {
#define CGS_BFP(S)                                                                                              \
    do {                                                                                                        \
        const int64_t nb = std::min<int64_t>(n_tiles, resident_blocks(reinterpret_cast<const void*>(&k_blend_fwd<1, S, true>), 64));            \
        if (nb <= 0) return hipErrorInvalidValue;                                                               \
        hipLaunchKernelGGL((k_blend_fwd<1, S, true>), dim3((unsigned)nb), dim3(64), 0, st, d_desc, ranges,       \
                           inst_rec, rec, qbits, image, T_final, n_last, n_blend, cnt);                         \
    } while (0)
        if (n_blend) CGS_BFP(true); else CGS_BFP(false);
#undef CGS_BFP
        return hipGetLastError();
    }
#define CGS_BF(W, S) hipLaunchKernelGGL((k_blend_fwd<W, S, false>), dim3((unsigned)((n_tiles + W - 1) / W)), \
                                        dim3(W * 64), 0, st, d_desc, ranges, inst_rec, rec, qbits, image, T_final, \
                                        n_last, n_blend, cnt)
    if (n_blend) {
        if (wpb == 1) CGS_BF(1, true); else if (wpb == 2) CGS_BF(2, true); else CGS_BF(4, true);
    } else {
        if (wpb == 1) CGS_BF(1, false); else if (wpb == 2) CGS_BF(2, false); else CGS_BF(4, false);
    }
#undef CGS_BF
    return hipGetLastError();
}

}  // namespace cgs
