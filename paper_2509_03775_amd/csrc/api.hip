// C-ABI entry points of libcgs: host-side validation, workspace planning and
// the launch sequences of the forward and backward render, the standalone
// binning and codebook-reduction calls, and the L1 loss.  Nothing here
// allocates device memory or synchronises; every launch goes to the caller's
// stream.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "cgs_internal.h"

namespace cgs {

// launchers defined in the other translation units
hipError_t launch_preprocess(const BatchDesc*, int, int, int64_t, float4*, uint32_t*, uint2*, uint32_t*, uint32_t*,
                             uint32_t*, uint32_t*, uint32_t*, const ZeroSpans&, hipStream_t);
hipError_t launch_capacity(DevCounters*, int64_t, int64_t*, hipStream_t);
hipError_t launch_emit(const BatchDesc*, int64_t, const uint32_t*, const uint32_t*, const uint2*, const uint32_t*,
                       const DevCounters*, void*, bool, uint32_t*, hipStream_t);
hipError_t launch_plain_counts(const uint16_t*, int64_t, uint32_t*, hipStream_t);
hipError_t launch_emit_plain(const uint16_t*, const int32_t*, const uint32_t*, const uint32_t*, int64_t, int32_t,
                             int32_t, const DevCounters*, uint32_t*, uint32_t*, hipStream_t);
hipError_t launch_plain_keys(const uint32_t*, const uint32_t*, const uint32_t*, const DevCounters*, int64_t,
                             uint64_t*, uint32_t*, hipStream_t);
hipError_t launch_blend_fwd(const BatchDesc*, int64_t, int, bool, const uint32_t*, const uint32_t*, const float4*,
                            uint8_t*, float*, float*, int32_t*, int32_t*, DevCounters*, hipStream_t);
hipError_t launch_blend_bwd(const BatchDesc*, int64_t, int, bool, const uint32_t*, const uint32_t*, const float4*,
                            const uint8_t*, const uint32_t*, const uint32_t*, const float*, const float*,
                            const int32_t*, float*, uint2*, DevCounters*, hipStream_t);
hipError_t launch_slot_sum(const BatchDesc*, int64_t, const float*, const uint32_t*, const uint32_t*, const uint2*,
                           const uint32_t*, const uint32_t*, const uint2*, const DevCounters*, float*, uint32_t*,
                           uint32_t*, int64_t, hipStream_t);
hipError_t launch_chain(const BatchDesc*, int, int, int64_t, const float*, const uint32_t*, float*, uint32_t*,
                        const uint32_t*, const uint32_t*, const uint32_t*, float*, hipStream_t);
hipError_t launch_merge_rows(const BatchDesc*, int64_t, const uint32_t*, const uint32_t*, const float*, const float*,
                             const uint32_t*, hipStream_t);
hipError_t launch_row_keys(const BatchDesc*, int, int64_t, uint32_t*, hipStream_t);
hipError_t launch_reduce(const BatchDesc*, int, const float*, int64_t, int, int, int, const uint32_t*,
                         const uint32_t*, int64_t, int64_t, const uint32_t*, hipStream_t);
hipError_t launch_gather_keys(const int32_t*, const int32_t*, int64_t, uint32_t*, uint32_t*, hipStream_t);
hipError_t launch_copy_keys(const int32_t*, int64_t, uint32_t*, hipStream_t);
hipError_t launch_l1(const float*, const float*, int64_t, float*, float*, float*, int, hipStream_t);
hipError_t launch_loss_recon(const LossViews&, const float*, const float*, float, float*, float*, float*, double*,
                             hipStream_t);
hipError_t launch_normals(int64_t, uint64_t, uint32_t, uint32_t, uint64_t, float*, uint32_t*, hipStream_t);
size_t mh_workspace(int64_t, int64_t, int64_t, int64_t, MhWs*, char*);
hipError_t mh_split(const MhArgs&, const MhWs&, hipStream_t);
hipError_t mh_merge(const MhArgs&, const MhWs&, hipStream_t);
int mh_transition_host(uint64_t, uint32_t);

namespace {

// Byte offsets of the forward/backward workspace arrays (host-side plan).
struct WsPlan {
    size_t desc, counters;
    size_t rec, depth_key, tile_rect, ntiles, prect, pay[2];
    size_t dsort_key[2], dsort_val[2];
    size_t offs, rect_d, cnt_d;
    size_t inst_key[2], inst_val[2];
    size_t tile_range, tile_cut, qbits, tperm_key[2], tperm_val[2];
    size_t radix_ws, radix_ws_tile, radix_ws_tlen, radix_ws_rows, scan_bsum, scan_bsum2;
    size_t chunk_tot, krange, chunk_base, ginst, rec_grad, rec_flag, isl_flag, gtheta, rpart, psort_key[2], psort_val[2], row_start;
    size_t total;
    int64_t scan_blocks_max;
};

int bits_for(int64_t n) {   // bits needed for values in [0, n)
    int b = 1;
    while (b < 40 && ((int64_t)1 << b) < n) ++b;
    return b;
}

int passes_for(int nbits) { return (nbits + kRadixBits - 1) / kRadixBits; }

// Bits of the heavy-first tile sort key (k_tile_len_keys writes 255 - q(length)).
constexpr int kTileLenKeyBits = 8;

template <typename T>
T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

struct Host {
    BatchDesc d;
    WsPlan p;
    int wpb;
    bool persist;
    int inst_buf;          // buffer pair holding the tile-sorted instances
    int dsort_buf;         // buffer pair holding the depth-sorted records
    int tile_bits;
    int tperm_buf;         // buffer pair holding the heavy-first tile order
    bool fused;            // every scene uses the single-codebook layout
    hipEvent_t* events;    // optional stage events
    int32_t* n_blend;      // optional per-pixel blended count
    int opacity_mode;
    int64_t rows_total;    // rows of the reduction key space (max of both parts)
};

size_t scan_bsum_count(int64_t n) { return (size_t)((n + kSortTile - 1) / kSortTile) + 16; }

cgs_status plan_batch(const cgs_batch* b, Host* h) {
    if (!b || !b->scenes || !b->cameras || !b->view_scene) return CGS_EINVAL;
    if (b->n_scenes < 1 || b->n_scenes > CGS_MAX_SCENES || b->n_views < 1 || b->n_views > CGS_MAX_VIEWS)
        return CGS_EINVAL;
    if (b->instance_capacity < 0 || b->instance_capacity >= ((int64_t)1 << 32)) return CGS_EINVAL;
    memset(&h->d, 0, sizeof(h->d));
    BatchDesc& d = h->d;
    d.n_views = b->n_views;
    d.n_scenes = b->n_scenes;
    d.capacity = b->instance_capacity;
    const cgs_scene& s0 = b->scenes[0];
    d.sh_degree = s0.sh_degree;
    d.dtype = s0.sr.dtype;
    if (s0.sh_degree < 0) return CGS_EINVAL;
    if (s0.sh_degree > 3) return CGS_EUNSUPPORTED;
    const int nco = (s0.sh_degree + 1) * (s0.sh_degree + 1);
    d.row_width = 8 + 3 * nco;
    h->opacity_mode = s0.opacity_mode;
    h->fused = true;
    int64_t goff = 0, sroff = 0, shoff = 0, gwaves = 0;
    for (int s = 0; s < b->n_scenes; ++s) {
        const cgs_scene& sc = b->scenes[s];
        if (sc.n < 0) return CGS_EINVAL;
        if (sc.sh_degree != s0.sh_degree) return CGS_EINVAL;
        if (sc.sr.dtype != d.dtype || sc.sh.dtype != d.dtype) return CGS_EINVAL;
        if (d.dtype != CGS_F32 && d.dtype != CGS_BF16) return CGS_EINVAL;
        if (sc.opacity_mode != 0 && sc.opacity_mode != 1) return CGS_EINVAL;
        if (sc.opacity_mode != h->opacity_mode) return CGS_EINVAL;
        if (sc.sr.rows <= 0 || sc.sh.rows <= 0) return CGS_EINVAL;
        if (!sc.sr.ptr || !sc.sh.ptr) return CGS_EINVAL;
        const int srcols = sc.opacity_mode ? 8 : 7;
        if (sc.sr.col0 < 0 || sc.sh.col0 < 0 || sc.sr.row_stride < sc.sr.col0 + srcols ||
            sc.sh.row_stride < sc.sh.col0 + 3 * nco)
            return CGS_EINVAL;
        if (sc.n > 0 && (!sc.means || !sc.idx_sr || !sc.idx_sh)) return CGS_EINVAL;
        if (sc.n > 0 && sc.opacity_mode == 0 && !sc.opacity_logit) return CGS_EINVAL;
        SceneDesc& sd = d.scenes[s];
        sd.n = sc.n;
        sd.g_off = goff;
        sd.wave_off = gwaves;
        gwaves += (sc.n + kWave - 1) / kWave;
        sd.sr_rows = sc.sr.rows;
        sd.sh_rows = sc.sh.rows;
        sd.sr_row_off = sroff;
        sd.sh_row_off = shoff;
        sd.means = sc.means;
        sd.idx_sr = sc.idx_sr;
        sd.idx_sh = sc.idx_sh;
        sd.sr = sc.sr.ptr;
        sd.sh = sc.sh.ptr;
        sd.opacity = sc.opacity_logit;
        sd.sr_stride = sc.sr.row_stride;
        sd.sr_col0 = sc.sr.col0;
        sd.sh_stride = sc.sh.row_stride;
        sd.sh_col0 = sc.sh.col0;
        sd.opacity_mode = sc.opacity_mode;
        sd.fused = (sc.idx_sr == sc.idx_sh && sc.sr.ptr == sc.sh.ptr && sc.sr.row_stride == sc.sh.row_stride &&
                    sc.sh.col0 == sc.sr.col0 + 8 && sc.opacity_mode == 1 && sc.sr.rows == sc.sh.rows) ? 1 : 0;
        if (!sd.fused) h->fused = false;
        goff += sc.n;
        sroff += sc.sr.rows;
        shoff += sc.sh.rows;
    }
    d.n_gauss = goff;
    d.n_gauss_waves = gwaves;
    {   // 16-byte vector loads of whole rows: degree-3 rows, opacity in the SR row, aligned windows
        const size_t esz = d.dtype == CGS_BF16 ? 2 : 4;
        bool vec = s0.sh_degree == 3 && h->opacity_mode == 1;
        for (int s = 0; s < b->n_scenes && vec; ++s) {
            const cgs_scene& sc = b->scenes[s];
            const uintptr_t a0 = reinterpret_cast<uintptr_t>(sc.sr.ptr) + esz * (size_t)sc.sr.col0;
            const uintptr_t a1 = reinterpret_cast<uintptr_t>(sc.sh.ptr) + esz * (size_t)sc.sh.col0;
            vec = (a0 % 16 == 0) && (a1 % 16 == 0) && ((esz * (size_t)sc.sr.row_stride) % 16 == 0) &&
                  ((esz * (size_t)sc.sh.row_stride) % 16 == 0);
        }
        d.vec_rows = vec ? 1 : 0;
    }
    d.sr_rows_total = sroff;
    d.sh_rows_total = shoff;
    if (goff >= ((int64_t)1 << 32) || sroff >= ((int64_t)1 << 32) || shoff >= ((int64_t)1 << 32)) return CGS_EINVAL;
    h->rows_total = std::max(sroff, shoff);
    int64_t roff = 0, toff = 0, poff = 0, rwaves = 0;
    d.pack_rect = 1;
    for (int v = 0; v < b->n_views; ++v) {
        const cgs_camera& c = b->cameras[v];
        const int s = b->view_scene[v];
        if (s < 0 || s >= b->n_scenes) return CGS_EINVAL;
        if (c.width <= 0 || c.height <= 0 || c.width > 65535 * kTile || c.height > 65535 * kTile) return CGS_EINVAL;
        if (!(c.fx > 0.f) || !(c.fy > 0.f)) return CGS_EINVAL;
        ViewDesc& vd = d.views[v];
        vd.W = c.width;
        vd.H = c.height;
        vd.tiles_x = (c.width + kTile - 1) / kTile;
        vd.tiles_y = (c.height + kTile - 1) / kTile;
        if (vd.tiles_x > 255 || vd.tiles_y > 255) d.pack_rect = 0;
        vd.scene = s;
        vd.tile_off = toff;
        vd.pix_off = poff;
        vd.rec_off = roff;
        vd.rec_wave_off = rwaves;
        rwaves += (b->scenes[s].n + kWave - 1) / kWave;
        vd.fx = c.fx; vd.fy = c.fy; vd.cx = c.cx; vd.cy = c.cy;
        {   // each step rounded to FP32, the device's order
            const volatile float hx = 0.5f * (float)c.width, hy = 0.5f * (float)c.height;
            const volatile float qx = hx / c.fx, qy = hy / c.fy;
            vd.limx = kClampFov * qx;
            vd.limy = kClampFov * qy;
        }
        memcpy(vd.Rt, c.Rt, sizeof(vd.Rt));
        memcpy(vd.campos, c.campos, sizeof(vd.campos));
        memcpy(vd.bg, c.bg, sizeof(vd.bg));
        roff += b->scenes[s].n;
        toff += (int64_t)vd.tiles_x * vd.tiles_y;
        poff += (int64_t)c.width * c.height;
    }
    d.n_rec = roff;
    d.n_rec_waves = rwaves;
    d.n_tiles = toff;
    d.n_pix = poff;
    if (roff >= ((int64_t)1 << 32) || toff >= ((int64_t)1 << 31)) return CGS_EINVAL;
    int nv = 0;
    for (int s = 0; s < b->n_scenes; ++s) {
        d.scenes[s].vfirst = nv;
        for (int v = 0; v < b->n_views; ++v)
            if (b->view_scene[v] == s) d.view_list[nv++] = v;
        d.scenes[s].vcount = nv - d.scenes[s].vfirst;
        for (int k = d.scenes[s].vfirst; k < nv; ++k) d.views[d.view_list[k]].scene_vi = k - d.scenes[s].vfirst;
    }
    {   // Gaussian-major flag offsets (the same total as the view-major record wavefronts)
        int64_t fw = 0;
        for (int s = 0; s < b->n_scenes; ++s) {
            SceneDesc& sd = d.scenes[s];
            sd.flag_wave_off = fw;
            fw += (sd.n + kWave - 1) / kWave * sd.vcount;
        }
        if (fw != d.n_rec_waves) return CGS_EINVAL;
    }
    const cgs_schedule* sch = b->schedule;
    h->wpb = (sch && (sch->blend_waves_per_block == 2 || sch->blend_waves_per_block == 4)) ? sch->blend_waves_per_block
                                                                                            : 1;
    d.tile_order = sch ? sch->tile_order : 0;
    if (d.tile_order < 0 || d.tile_order > 2) return CGS_EINVAL;
    if (sch && (sch->persistent < 0 || sch->persistent > 1)) return CGS_EINVAL;
    h->persist = sch && sch->persistent == 1;
    if (h->persist) h->wpb = 1;
    h->events = sch ? reinterpret_cast<hipEvent_t*>(sch->stage_events) : nullptr;
    h->n_blend = sch ? sch->n_blend : nullptr;
    h->tile_bits = bits_for(d.n_tiles);
    h->inst_buf = (passes_for(h->tile_bits) - 1) & 1;
    h->tperm_buf = (passes_for(kTileLenKeyBits) - 1) & 1;
    h->dsort_buf = (passes_for(31) - 1) & 1;

    // workspace plan
    WsPlan& p = h->p;
    const int64_t R = d.n_rec, G = d.n_gauss, cap = d.capacity, T = d.n_tiles;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    p.desc = take(sizeof(BatchDesc));
    p.counters = take(sizeof(DevCounters));
    p.rec = take(16 * kRecF4 * (size_t)R);
    p.depth_key = take(4 * (size_t)R);
    p.tile_rect = take(8 * (size_t)R);
    p.ntiles = take(4 * (size_t)R);
    p.prect = take(4 * (size_t)R);
    for (int i = 0; i < 2; ++i) p.pay[i] = take(4 * (size_t)R);
    for (int i = 0; i < 2; ++i) { p.dsort_key[i] = take(4 * (size_t)R); p.dsort_val[i] = take(4 * (size_t)R); }
    p.offs = take(4 * (size_t)R);
    p.rect_d = take(8 * (size_t)R);
    p.cnt_d = take(4 * (size_t)R);
    for (int i = 0; i < 2; ++i) { p.inst_key[i] = take(4 * (size_t)cap); p.inst_val[i] = take(4 * (size_t)cap); }
    p.tile_range = take(8 * (size_t)T);
    p.tile_cut = take(8 * (size_t)T);
    p.qbits = take((size_t)cap);
    for (int i = 0; i < 2; ++i) { p.tperm_key[i] = take(4 * (size_t)T); p.tperm_val[i] = take(4 * (size_t)T); }
    const int64_t nmax = std::max(std::max(R, cap), std::max(G, T));   // every sort and scan below
    p.radix_ws = take(radix_ws_bytes(nmax));
    p.radix_ws_rows = take(radix_ws_bytes(std::max<int64_t>(G, 1)));   // the row sort runs beside the forward's sorts
    // the tile sort and the tile-length sort have their own, so that the
    // preprocess can zero all three sorts' counters up front
    p.radix_ws_tile = take(radix_ws_bytes(std::max<int64_t>(cap, 1)));
    p.radix_ws_tlen = take(radix_ws_bytes(std::max<int64_t>(T, 1)));
    p.scan_blocks_max = (int64_t)scan_bsum_count(nmax);
    p.scan_bsum = take(8 * (size_t)p.scan_blocks_max);
    p.scan_bsum2 = take(8 * (size_t)p.scan_blocks_max);
    p.chunk_tot = take(4 * (size_t)d.n_rec_waves + 4);
    p.krange = take(8 * (size_t)d.n_rec_waves + 8);
    p.chunk_base = take(4 * (size_t)d.n_rec_waves + 4);
    p.ginst = take(4 * 9 * (size_t)cap);
    p.rec_grad = take(4 * 9 * (size_t)R);
    p.rec_flag = take(32 * (size_t)d.n_rec_waves + 32);
    p.isl_flag = take(8 * (size_t)d.n_gauss_waves + 8);
    p.gtheta = take(4 * (size_t)d.row_width * (size_t)G);
    p.rpart = take(4 * (size_t)d.row_width * 2 * (size_t)d.n_gauss_waves);    // head and tail partial per wavefront
    for (int i = 0; i < 2; ++i) { p.psort_key[i] = take(4 * (size_t)G); p.psort_val[i] = take(4 * (size_t)G); }
    p.row_start = take(8 * (size_t)(h->rows_total + 1));
    p.total = o;
    return CGS_OK;
}

cgs_status hip_status(hipError_t e) { return e == hipSuccess ? CGS_OK : CGS_EHIP; }

#define CGS_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return CGS_EHIP;          \
    } while (0)

// Upload the used part of the descriptor (header + views, then scenes).
hipError_t upload_desc(const Host& h, void* ws, hipStream_t st) {
    char* base = static_cast<char*>(ws) + h.p.desc;
    const size_t head = offsetof(BatchDesc, views) + sizeof(ViewDesc) * (size_t)h.d.n_views;
    const size_t so = offsetof(BatchDesc, scenes);
    return upload_two(base, &h.d, head, base + so, reinterpret_cast<const char*>(&h.d) + so,
                      sizeof(SceneDesc) * (size_t)h.d.n_scenes, st);
}

hipError_t mark(const Host& h, int i, hipStream_t st) {
    return h.events ? hipEventRecord(h.events[i], st) : hipSuccess;
}

// A second stream per device for work that does not depend on the kernels
// just before it on the caller's stream.  Created on first use (default
// priority, non-blocking) with two events and kept until the process ends;
// work is forked to it and joined back by events, so the caller's stream
// still orders everything and a graph capture follows the dependencies.  It
// is not created while the caller's stream is being captured (the work then
// stays on the caller's stream), and calls that use it are serialised per
// device from fork to join.
struct Side {
    std::mutex mu;
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool failed = false;
};

Side* side_stream(hipStream_t caller) {
    static Side sides[64];
    static std::mutex create_mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    Side& sd = sides[dev];
    std::lock_guard<std::mutex> lk(create_mu);
    if (sd.s || sd.failed) return sd.s ? &sd : nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(caller, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    if (hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sd.join, hipEventDisableTiming) != hipSuccess) {
        sd.failed = true;
        sd.s = nullptr;
        return nullptr;
    }
    return &sd;
}

// Fork: the side stream waits for everything enqueued on `st` so far.
hipError_t side_fork(Side* sd, hipStream_t st) {
    hipError_t e = hipEventRecord(sd->fork, st);
    return e == hipSuccess ? hipStreamWaitEvent(sd->s, sd->fork, 0) : e;
}

// Join: `st` waits for everything enqueued on the side stream so far.
hipError_t side_join(Side* sd, hipStream_t st) {
    hipError_t e = hipEventRecord(sd->join, sd->s);
    return e == hipSuccess ? hipStreamWaitEvent(st, sd->join, 0) : e;
}

// Joins the side stream back into the caller's stream when a call returns
// early (an error after the fork), so no forked work is left outside the
// caller's stream order or a capture of it.  The normal path joins
// explicitly with join(), which reports the join's own error.
struct SideGuard {
    Side* sd = nullptr;
    hipStream_t st = nullptr;
    hipError_t join() {
        Side* s = sd;
        sd = nullptr;
        return s ? side_join(s, st) : hipSuccess;
    }
    ~SideGuard() {
        if (sd) (void)side_join(sd, st);
    }
};

// Device scratch of cgs_codebook_grad_reduce_noalloc (its workspace): one
// copy per device, loaded with the library's code and held until the process
// ends.  Host code never passes `scratch` itself (on the host it is only a
// stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

void* noalloc_scratch() {
    static void* addr[64];
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        addr[dev] = p;
    }
    return addr[dev];
}

}  // namespace
}  // namespace cgs

using namespace cgs;

extern "C" {

int32_t cgs_version(void) { return 10000; }

uint32_t cgs_sort_stalls(void) { return sort_stalls(); }

const char* cgs_status_str(int32_t s) {
    switch (s) {
        case CGS_OK: return "ok";
        case CGS_EINVAL: return "invalid argument";
        case CGS_EUNSUPPORTED: return "unsupported option";
        case CGS_ECAPACITY: return "instance capacity exceeded";
        case CGS_EHIP: return "HIP launch failed";
        case CGS_EWORKSPACE: return "workspace too small";
        case CGS_ELIMIT: return "sizes exceed the fixed device scratch of the allocation-free call";
        default: return "unknown status";
    }
}

size_t cgs_workspace_bytes(const cgs_batch* batch) {
    static thread_local Host h;
    if (plan_batch(batch, &h) != CGS_OK) return 0;
    return h.p.total;
}

cgs_status cgs_workspace_layout(const cgs_batch* batch, cgs_ws_layout* out) {
    static thread_local Host h;
    cgs_status s = plan_batch(batch, &h);
    if (s != CGS_OK) return s;
    if (!out) return CGS_EINVAL;
    out->records = h.p.rec;
    out->depth_key = h.p.depth_key;
    out->tile_rect = h.p.tile_rect;
    out->inst_rec = h.p.inst_val[h.inst_buf];
    out->tile_range = h.p.tile_range;
    out->n_records = h.d.n_rec;
    out->n_tiles = h.d.n_tiles;
    return CGS_OK;
}

// Buffer of the Gaussians' row order (psort_key/val[b]) after the forward's
// row sort: the last of its 8-bit passes writes buffer (passes - 1) & 1.
int row_sort_buf(const Host& h) { return (passes_for(bits_for(h.d.sr_rows_total)) - 1) & 1; }

// The Gaussians sorted by codebook row (single-codebook layout: the SR and
// SH rows are the same), and each row's range of the sorted order.
hipError_t sort_rows(const Host& h, void* ws, const BatchDesc* dd, hipStream_t s2) {
    const WsPlan& p = h.p;
    uint32_t* pk[2] = {at<uint32_t>(ws, p.psort_key[0]), at<uint32_t>(ws, p.psort_key[1])};
    uint32_t* pv[2] = {at<uint32_t>(ws, p.psort_val[0]), at<uint32_t>(ws, p.psort_val[1])};
    hipError_t e = launch_row_keys(dd, 0, h.d.n_gauss, pk[1], s2);
    if (e != hipSuccess) return e;
    const int pb = radix_sort_pairs(pk[1], nullptr, pk, pv, h.d.n_gauss, nullptr, bits_for(h.d.sr_rows_total),
                                    at<char>(ws, p.radix_ws_rows), s2, &e);
    if (e != hipSuccess) return e;
    if (pb != row_sort_buf(h)) return hipErrorUnknown;
    return tile_ranges(pk[pb], nullptr, h.d.n_gauss, h.d.sr_rows_total, at<uint32_t>(ws, p.row_start), s2);
}

cgs_status cgs_render_forward(const cgs_batch* batch, float* image, float* T_final, int32_t* n_last, void* ws,
                              size_t ws_bytes, int64_t* d_info, void* stream) {
    static thread_local Host h;
    cgs_status s = plan_batch(batch, &h);
    if (s != CGS_OK) return s;
    if (!ws) return CGS_EINVAL;
    if (ws_bytes < h.p.total) return CGS_EWORKSPACE;
    if (h.d.n_pix > 0 && (!image || !T_final || !n_last)) return CGS_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const WsPlan& p = h.p;
    const BatchDesc* dd = at<const BatchDesc>(ws, p.desc);
    DevCounters* cnt = at<DevCounters>(ws, p.counters);
    unsigned long long* bsum = at<unsigned long long>(ws, p.scan_bsum);
    void* sws = at<char>(ws, p.radix_ws);
    CGS_TRY(mark(h, 0, st));
    h.d.tile_perm = at<const uint32_t>(ws, p.tperm_val[h.tperm_buf]);
    CGS_TRY(upload_desc(h, ws, st));
    // the preprocess zeroes the counters of the depth sort, the instance
    // offset scan, the tile sort and the tile-length sort (no fill launches)
    void* sws_tile = at<char>(ws, p.radix_ws_tile);
    void* sws_tlen = at<char>(ws, p.radix_ws_tlen);
    ZeroSpans zero{};
    zero.p[0] = sort_counters(sws, h.d.n_rec, &zero.n[0]);
    zero.p[1] = scan_states(bsum, h.d.n_rec, &zero.n[1]);
    zero.p[2] = sort_counters(sws_tile, h.d.capacity, &zero.n[2]);
    zero.p[3] = sort_counters(sws_tlen, h.d.n_tiles, &zero.n[3]);
    CGS_TRY(launch_preprocess(dd, h.d.dtype, h.d.sh_degree, h.d.n_gauss_waves, at<float4>(ws, p.rec), at<uint32_t>(ws, p.depth_key),
                              at<uint2>(ws, p.tile_rect), at<uint32_t>(ws, p.ntiles), at<uint32_t>(ws, p.prect),
                              at<uint32_t>(ws, p.chunk_tot), at<uint32_t>(ws, p.krange), at<uint32_t>(ws, p.rec_flag),
                              zero, st));
    CGS_TRY(mark(h, 1, st));
    // backward gradient slots: each 64-record chunk owns a contiguous range
    // (chunks in record order); its base, needed only by the backward, is
    // scanned from the chunk totals beside the depth sort on the side stream
    Side* side = side_stream(st);
    std::unique_lock<std::mutex> side_lk;
    SideGuard guard;        // declared after the lock: joins before it is released
    if (side) {
        side_lk = std::unique_lock<std::mutex>(side->mu);
        CGS_TRY(side_fork(side, st));
        guard.sd = side;
        guard.st = st;
    }
    CGS_TRY(scan_u32(at<uint32_t>(ws, p.chunk_tot), nullptr, h.d.n_rec_waves, at<uint32_t>(ws, p.chunk_base), nullptr,
                     at<unsigned long long>(ws, p.scan_bsum2), side ? side->s : st));
    // Single-codebook layout: the Gaussians in codebook-row order, which the
    // backward's fused chain rule and row reduction walk.  It depends only on
    // the indices, so it runs beside the binning on the side stream (inline
    // without one), with a sort workspace of its own.
    if (h.fused) CGS_TRY(sort_rows(h, ws, dd, side ? side->s : st));
    // depth order of every record (stable: ties keep record order)
    uint32_t* dk[2] = {at<uint32_t>(ws, p.dsort_key[0]), at<uint32_t>(ws, p.dsort_key[1])};
    uint32_t* dv[2] = {at<uint32_t>(ws, p.dsort_val[0]), at<uint32_t>(ws, p.dsort_val[1])};
    hipError_t e;
    // the depth-ordered tile rectangle and count of each record: carried
    // through the sort packed in one word when every view has fewer than 256
    // tiles per side, else gathered by the last pass
    SortGather rg{at<const uint2>(ws, p.tile_rect), at<uint2>(ws, p.rect_d), at<uint32_t>(ws, p.cnt_d), 1, nullptr,
                  {nullptr, nullptr}};
    if (h.d.pack_rect) {
        rg.pay_in = at<const uint32_t>(ws, p.prect);
        rg.pay_buf[0] = at<uint32_t>(ws, p.pay[0]);
        rg.pay_buf[1] = at<uint32_t>(ws, p.pay[1]);
    }
    const int db = h.d.pack_rect
                       ? radix_sort_depth(at<uint32_t>(ws, p.depth_key), at<uint32_t>(ws, p.krange), h.d.n_rec_waves,
                                          dk, dv, h.d.n_rec, sws, st, &e, rg, true)
                       : radix_sort_pairs(at<uint32_t>(ws, p.depth_key), nullptr, dk, dv, h.d.n_rec, nullptr, 31, sws,
                                          st, &e, &rg, true);
    CGS_TRY(e);
    // instance offsets in depth order, capacity check, emission
    CGS_TRY(scan_u32(at<uint32_t>(ws, p.cnt_d), nullptr, h.d.n_rec, at<uint32_t>(ws, p.offs), &cnt->n_inst, bsum, st,
                     true));
    CGS_TRY(launch_capacity(cnt, h.d.capacity, d_info, st));
    uint32_t* ik[2] = {at<uint32_t>(ws, p.inst_key[0]), at<uint32_t>(ws, p.inst_key[1])};
    uint32_t* iv[2] = {at<uint32_t>(ws, p.inst_val[0]), at<uint32_t>(ws, p.inst_val[1])};
    // tile keys stored in 16 bits when the batch has at most 65536 tiles
    const bool key16 = h.tile_bits <= 16;
    CGS_TRY(launch_emit(dd, h.d.n_rec, dv[db], at<uint32_t>(ws, p.offs), at<uint2>(ws, p.rect_d),
                        at<uint32_t>(ws, p.cnt_d), cnt, ik[1], key16, iv[1], st));
    int ib;
    if (key16) {
        uint16_t* ik16[2] = {reinterpret_cast<uint16_t*>(ik[0]), reinterpret_cast<uint16_t*>(ik[1])};
        ib = radix_sort_pairs16(ik16[1], iv[1], ik16, iv, h.d.capacity, &cnt->n_inst_ok, h.tile_bits, sws_tile, st, &e,
                                true);
        CGS_TRY(e);
        if (ib != h.inst_buf) return CGS_EHIP;
        CGS_TRY(tile_ranges16(ik16[ib], &cnt->n_inst_ok, h.d.capacity, h.d.n_tiles, at<uint32_t>(ws, p.tile_range),
                              st));
    } else {
        ib = radix_sort_pairs(ik[1], iv[1], ik, iv, h.d.capacity, &cnt->n_inst_ok, h.tile_bits, sws_tile, st, &e,
                              nullptr, true);
        CGS_TRY(e);
        if (ib != h.inst_buf) return CGS_EHIP;
        CGS_TRY(tile_ranges(ik[ib], &cnt->n_inst_ok, h.d.capacity, h.d.n_tiles, at<uint32_t>(ws, p.tile_range), st));
    }
    if (h.d.tile_order == 2) {
        uint32_t* tk[2] = {at<uint32_t>(ws, p.tperm_key[0]), at<uint32_t>(ws, p.tperm_key[1])};
        uint32_t* tv[2] = {at<uint32_t>(ws, p.tperm_val[0]), at<uint32_t>(ws, p.tperm_val[1])};
        CGS_TRY(tile_len_keys(at<uint32_t>(ws, p.tile_range), h.d.n_tiles, tk[1], st));
        const int tb = radix_sort_pairs(tk[1], nullptr, tk, tv, h.d.n_tiles, nullptr, kTileLenKeyBits, sws_tlen, st, &e,
                                        nullptr, true);
        CGS_TRY(e);
        if (tb != h.tperm_buf) return CGS_EHIP;
    }
    CGS_TRY(mark(h, 2, st));
    CGS_TRY(launch_blend_fwd(dd, h.d.n_tiles, h.wpb, h.persist, at<uint32_t>(ws, p.tile_range), iv[ib],
                             at<float4>(ws, p.rec), at<uint8_t>(ws, p.qbits), image, T_final, n_last, h.n_blend, cnt,
                             st));
    CGS_TRY(guard.join());
    CGS_TRY(mark(h, 3, st));
    return CGS_OK;
}

namespace {

// Backward shared by the plain entry point and the one with the fused SGLD
// update (sgld and params both NULL: gradients only).
cgs_status backward_impl(const cgs_batch* batch, const float* grad_image, const float* T_final, const int32_t* n_last,
                         const cgs_scene_grads* grads, const cgs_sgld* sgld, const cgs_scene_params* params, void* ws,
                         size_t ws_bytes, void* stream) {
    static thread_local Host h;
    cgs_status s = plan_batch(batch, &h);
    if (s != CGS_OK) return s;
    if (!ws || !grads) return CGS_EINVAL;
    h.d.sgld = 0;
    if (sgld) {
        if (!params) return CGS_EINVAL;
        for (int k = 0; k < 4; ++k) {
            const float e = (&sgld->eps_means)[k];
            if (!(e >= 0.f) || !(e < 3.0e38f)) return CGS_EINVAL;
            h.d.eps[k] = e;
        }
        h.d.sgld = 1;
        h.d.seed = sgld->seed;
        h.d.step = (int32_t)sgld->step;
        const int nco = (h.d.row_width - 8) / 3;
        for (int i = 0; i < batch->n_scenes; ++i) {
            const cgs_scene_params& q = params[i];
            SceneDesc& sd = h.d.scenes[i];
            if (sd.n > 0 && !q.means) return CGS_EINVAL;
            if (h.opacity_mode == 0 && sd.n > 0 && !q.opacity_logit) return CGS_EINVAL;
            if (!q.sr || !q.sh) return CGS_EINVAL;
            if (q.sr_col0 < 0 || q.sr_stride < q.sr_col0 + (h.opacity_mode ? 8 : 7)) return CGS_EINVAL;
            if (q.sh_col0 < 0 || q.sh_stride < q.sh_col0 + 3 * nco) return CGS_EINVAL;
            sd.u_means = q.means;
            sd.u_opacity = q.opacity_logit;
            sd.u_sr = q.sr;
            sd.u_sr_stride = q.sr_stride;
            sd.u_sr_col0 = q.sr_col0;
            sd.u_sh = q.sh;
            sd.u_sh_stride = q.sh_stride;
            sd.u_sh_col0 = q.sh_col0;
        }
    }
    if (ws_bytes < h.p.total) return CGS_EWORKSPACE;
    if (h.d.n_pix > 0 && (!grad_image || !T_final || !n_last)) return CGS_EINVAL;
    bool single = h.fused;
    for (int i = 0; i < batch->n_scenes; ++i) {
        const cgs_scene_grads& g = grads[i];
        SceneDesc& sd = h.d.scenes[i];
        if (sd.n > 0 && !g.means) return CGS_EINVAL;
        if (!g.sr || (!g.sh && !sd.fused)) return CGS_EINVAL;
        const int srcols = h.opacity_mode ? 8 : 7;
        if (g.sr_col0 < 0 || g.sr_stride < g.sr_col0 + srcols) return CGS_EINVAL;
        if (g.sh && (g.sh_col0 < 0 || g.sh_stride < g.sh_col0 + h.d.row_width - 8)) return CGS_EINVAL;
        if (h.opacity_mode == 0 && sd.n > 0 && !g.opacity) return CGS_EINVAL;
        sd.g_means = g.means;
        sd.g_sr = g.sr;
        sd.g_sr_stride = g.sr_stride;
        sd.g_sr_col0 = g.sr_col0;
        sd.g_sh = g.sh ? g.sh : g.sr;
        sd.g_sh_stride = g.sh ? g.sh_stride : g.sr_stride;
        sd.g_sh_col0 = g.sh ? g.sh_col0 : g.sr_col0 + 8;
        sd.g_opacity = g.opacity;
        if (!(sd.g_sh == sd.g_sr && sd.g_sh_stride == sd.g_sr_stride && sd.g_sh_col0 == sd.g_sr_col0 + 8))
            single = false;
        if (!sd.fused && g.sr_stride < g.sr_col0 + srcols) return CGS_EINVAL;
        if (single && g.sr_stride < g.sr_col0 + h.d.row_width) return CGS_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const WsPlan& p = h.p;
    const BatchDesc* dd = at<const BatchDesc>(ws, p.desc);
    void* sws = at<char>(ws, p.radix_ws);
    DevCounters* cnt = at<DevCounters>(ws, p.counters);
    h.d.tile_perm = at<const uint32_t>(ws, p.tperm_val[h.tperm_buf]);
    CGS_TRY(upload_desc(h, ws, st));
    CGS_TRY(mark(h, 4, st));
    uint32_t* pk[2] = {at<uint32_t>(ws, p.psort_key[0]), at<uint32_t>(ws, p.psort_key[1])};
    uint32_t* pv[2] = {at<uint32_t>(ws, p.psort_val[0]), at<uint32_t>(ws, p.psort_val[1])};
    uint32_t* rr = at<uint32_t>(ws, p.row_start);
    // the two-codebook layout sorts the Gaussians by each codebook's rows here
    auto sort_part = [&](int part_i, int64_t rows, int* pb) -> hipError_t {
        hipError_t e = launch_row_keys(dd, part_i, h.d.n_gauss, pk[1], st);
        if (e != hipSuccess) return e;
        *pb = radix_sort_pairs(pk[1], nullptr, pk, pv, h.d.n_gauss, nullptr, bits_for(rows), sws, st, &e);
        if (e != hipSuccess) return e;
        return tile_ranges(pk[*pb], nullptr, h.d.n_gauss, rows, rr, st);
    };
    float* ginst = at<float>(ws, p.ginst);
    CGS_TRY(launch_blend_bwd(dd, h.d.n_tiles, h.wpb, h.persist, at<uint32_t>(ws, p.tile_range),
                             at<uint32_t>(ws, p.inst_val[h.inst_buf]),
                             at<float4>(ws, p.rec), at<const uint8_t>(ws, p.qbits), at<uint32_t>(ws, p.depth_key),
                             at<uint32_t>(ws, p.chunk_base),
                             grad_image, T_final, n_last, ginst, at<uint2>(ws, p.tile_cut), cnt, st));
    CGS_TRY(mark(h, 5, st));
    float* gth = at<float>(ws, p.gtheta);
    float* rgrad = at<float>(ws, p.rec_grad);
    uint32_t* rflag = at<uint32_t>(ws, p.rec_flag);
    uint32_t* islf = at<uint32_t>(ws, p.isl_flag);
    CGS_TRY(launch_slot_sum(dd, h.d.n_rec_waves, ginst, at<uint32_t>(ws, p.chunk_base), at<uint32_t>(ws, p.ntiles),
                            at<uint2>(ws, p.tile_rect), at<uint32_t>(ws, p.prect), at<uint32_t>(ws, p.depth_key),
                            at<uint2>(ws, p.tile_cut), cnt, rgrad, rflag, islf, h.d.n_gauss_waves, st));
    if (single) {
        // Single codebook: the chain rule walks the Gaussians in row order and
        // reduces the rows itself, in the order the forward sorted (the
        // indices are the forward's: a backward follows its forward)
        const int pb = row_sort_buf(h);
        CGS_TRY(launch_chain(dd, h.d.dtype, h.d.sh_degree, h.d.n_gauss_waves, rgrad, rflag, gth, islf,
                             pk[pb], pv[pb], rr, at<float>(ws, p.rpart), st));
        CGS_TRY(mark(h, 6, st));
        CGS_TRY(launch_merge_rows(dd, h.d.sr_rows_total, pv[pb], rr, at<float>(ws, p.rpart), gth, islf, st));
    } else {
        CGS_TRY(launch_chain(dd, h.d.dtype, h.d.sh_degree, h.d.n_gauss_waves, rgrad, rflag, gth, islf,
                             nullptr, nullptr, nullptr, nullptr, st));
        CGS_TRY(mark(h, 6, st));
        for (int part_i = 0; part_i < 2; ++part_i) {
            const int64_t rows = part_i == 0 ? h.d.sr_rows_total : h.d.sh_rows_total;
            const int c0 = part_i == 0 ? 0 : 8;
            const int D = part_i == 0 ? (h.opacity_mode ? 8 : 7) : h.d.row_width - 8;
            int pb = 0;
            CGS_TRY(sort_part(part_i, rows, &pb));
            CGS_TRY(launch_reduce(dd, part_i, gth, h.d.row_width, c0, D, 0, pk[pb], pv[pb], h.d.n_gauss, rows, rr, st));
        }
    }
    CGS_TRY(mark(h, 7, st));
    return CGS_OK;
}

}  // namespace

cgs_status cgs_render_backward(const cgs_batch* batch, const float* grad_image, const float* T_final,
                               const int32_t* n_last, const cgs_scene_grads* grads, void* ws, size_t ws_bytes,
                               int64_t* d_info, void* stream) {
    (void)d_info;
    return backward_impl(batch, grad_image, T_final, n_last, grads, nullptr, nullptr, ws, ws_bytes, stream);
}

cgs_status cgs_render_backward_sgld(const cgs_batch* batch, const float* grad_image, const float* T_final,
                                    const int32_t* n_last, const cgs_scene_grads* grads, const cgs_sgld* sgld,
                                    const cgs_scene_params* params, void* ws, size_t ws_bytes, int64_t* d_info,
                                    void* stream) {
    (void)d_info;
    if (!sgld || !params) return CGS_EINVAL;
    return backward_impl(batch, grad_image, T_final, n_last, grads, sgld, params, ws, ws_bytes, stream);
}

size_t cgs_codebook_grad_reduce_workspace_bytes(int64_t n, int64_t k, int32_t d) {
    if (n < 0 || k <= 0 || d <= 0) return 0;
    size_t o = 0;
    auto take = [&](size_t bytes) { o = align_up(o + bytes); };
    take(sizeof(BatchDesc));
    for (int i = 0; i < 4; ++i) take(4 * (size_t)n);
    take(8 * (size_t)(k + 1));
    take(radix_ws_bytes(n));
    return o;
}

cgs_status cgs_codebook_grad_reduce(const float* g, int64_t ld, const int32_t* idx, const int32_t* perm, int64_t n,
                                    int64_t k, int32_t d, float* grad_cb, int64_t ld_out, void* ws, size_t ws_bytes,
                                    void* stream) {
    if (n < 0 || k <= 0 || d <= 0 || ld < d || ld_out < d) return CGS_EINVAL;
    if (k >= ((int64_t)1 << 32) || n >= ((int64_t)1 << 32)) return CGS_EINVAL;
    if (!grad_cb || !ws || (n > 0 && (!g || !idx))) return CGS_EINVAL;
    const size_t need = cgs_codebook_grad_reduce_workspace_bytes(n, k, d);
    if (ws_bytes < need) return CGS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    static thread_local BatchDesc hd;
    memset(&hd, 0, offsetof(BatchDesc, views));
    hd.n_scenes = 1;
    hd.n_gauss = n;
    hd.sr_rows_total = k;
    SceneDesc sd;
    memset(&sd, 0, sizeof(sd));
    sd.n = n;
    sd.sr_rows = k;
    sd.g_sr = grad_cb;
    sd.g_sr_stride = (int32_t)ld_out;
    sd.g_sr_col0 = 0;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    const size_t o_desc = take(sizeof(BatchDesc));
    uint32_t* pk[2];
    uint32_t* pv[2];
    for (int i = 0; i < 2; ++i) { pk[i] = at<uint32_t>(ws, take(4 * (size_t)n)); pv[i] = at<uint32_t>(ws, take(4 * (size_t)n)); }
    uint32_t* rr = at<uint32_t>(ws, take(8 * (size_t)(k + 1)));
    void* sws = at<char>(ws, take(radix_ws_bytes(n)));
    char* dbase = static_cast<char*>(ws) + o_desc;
    CGS_TRY(upload_bytes(dbase, &hd, offsetof(BatchDesc, views), st));
    CGS_TRY(upload_bytes(dbase + offsetof(BatchDesc, scenes), &sd, sizeof(sd), st));
    const BatchDesc* dd = reinterpret_cast<const BatchDesc*>(dbase);
    int pb = 0;
    if (perm) {
        CGS_TRY(launch_gather_keys(idx, perm, n, pk[0], pv[0], st));
    } else {
        CGS_TRY(launch_copy_keys(idx, n, pk[1], st));
        hipError_t e;
        pb = radix_sort_pairs(pk[1], nullptr, pk, pv, n, nullptr, bits_for(k), sws, st, &e);
        CGS_TRY(e);
    }
    CGS_TRY(tile_ranges(pk[pb], nullptr, n, k, rr, st));
    CGS_TRY(launch_reduce(dd, 0, g, ld, 0, d, 0, pk[pb], pv[pb], n, k, rr, st));
    return CGS_OK;
}

cgs_status cgs_codebook_grad_reduce_noalloc(const float* g, int64_t ld, const int32_t* idx, const int32_t* perm,
                                            int64_t n, int64_t k, int32_t d, float* grad_cb, int64_t ld_out,
                                            void* stream) {
    const size_t need = cgs_codebook_grad_reduce_workspace_bytes(n, k, d);
    if (need == 0) return CGS_EINVAL;
    if (need > kNoAllocScratchBytes) return CGS_ELIMIT;
    void* ws = noalloc_scratch();
    if (!ws) return CGS_EHIP;
    return cgs_codebook_grad_reduce(g, ld, idx, perm, n, k, d, grad_cb, ld_out, ws, kNoAllocScratchBytes, stream);
}

size_t cgs_bin_tiles_workspace_bytes(int64_t n, int32_t tiles_x, int32_t tiles_y, int32_t n_views, int64_t capacity) {
    if (n < 0 || tiles_x <= 0 || tiles_y <= 0 || n_views <= 0 || capacity < 0) return 0;
    size_t o = 0;
    auto take = [&](size_t bytes) { o = align_up(o + bytes); };
    take(sizeof(DevCounters));
    for (int i = 0; i < 6; ++i) take(4 * (size_t)n);        // ntiles, offs, dsort key/val x2
    for (int i = 0; i < 4; ++i) take(4 * (size_t)capacity); // instance key/val x2
    const int64_t nmax = std::max(n, capacity);
    take(radix_ws_bytes(nmax));
    take(8 * scan_bsum_count(nmax));
    return o;
}

cgs_status cgs_bin_tiles(const uint32_t* depth_key, const uint16_t* trect, const int32_t* view_of, int64_t n,
                         int32_t tiles_x, int32_t tiles_y, int32_t n_views, uint64_t* sorted_key, uint32_t* sorted_gid,
                         uint32_t* tile_range, int64_t capacity, int64_t* d_info, void* ws, size_t ws_bytes,
                         void* stream) {
    if (n < 0 || tiles_x <= 0 || tiles_y <= 0 || n_views <= 0 || capacity < 0) return CGS_EINVAL;
    if (tiles_x > 65535 || tiles_y > 65535) return CGS_EINVAL;
    const int64_t ntile = (int64_t)tiles_x * tiles_y * n_views;
    if (ntile >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 32) || capacity >= ((int64_t)1 << 32)) return CGS_EINVAL;
    if (!ws || !sorted_gid || !tile_range || (n > 0 && (!depth_key || !trect))) return CGS_EINVAL;
    if (ws_bytes < cgs_bin_tiles_workspace_bytes(n, tiles_x, tiles_y, n_views, capacity)) return CGS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    DevCounters* cnt = at<DevCounters>(ws, take(sizeof(DevCounters)));
    uint32_t* nt = at<uint32_t>(ws, take(4 * (size_t)n));
    uint32_t* offs = at<uint32_t>(ws, take(4 * (size_t)n));
    uint32_t* dk[2];
    uint32_t* dv[2];
    for (int i = 0; i < 2; ++i) { dk[i] = at<uint32_t>(ws, take(4 * (size_t)n)); dv[i] = at<uint32_t>(ws, take(4 * (size_t)n)); }
    uint32_t* ik[2];
    uint32_t* iv[2];
    for (int i = 0; i < 2; ++i) {
        ik[i] = at<uint32_t>(ws, take(4 * (size_t)capacity));
        iv[i] = at<uint32_t>(ws, take(4 * (size_t)capacity));
    }
    const int64_t nmax = std::max(n, capacity);
    void* sws = at<char>(ws, take(radix_ws_bytes(nmax)));
    unsigned long long* bsum = at<unsigned long long>(ws, take(8 * scan_bsum_count(nmax)));
    CGS_TRY(launch_plain_counts(trect, n, nt, st));
    hipError_t e;
    int db = radix_sort_pairs(depth_key, nullptr, dk, dv, n, nullptr, 32, sws, st, &e);
    CGS_TRY(e);
    CGS_TRY(scan_u32(nt, dv[db], n, offs, &cnt->n_inst, bsum, st));
    CGS_TRY(launch_capacity(cnt, capacity, d_info, st));
    CGS_TRY(launch_emit_plain(trect, view_of, dv[db], offs, n, tiles_x, tiles_y, cnt, ik[1], iv[1], st));
    int ib = radix_sort_pairs(ik[1], iv[1], ik, iv, capacity, &cnt->n_inst_ok, bits_for(ntile), sws, st, &e);
    CGS_TRY(e);
    CGS_TRY(tile_ranges(ik[ib], &cnt->n_inst_ok, capacity, ntile, tile_range, st));
    CGS_TRY(launch_plain_keys(ik[ib], iv[ib], depth_key, cnt, capacity, sorted_key, sorted_gid, st));
    return CGS_OK;
}

size_t cgs_loss_l1_workspace_bytes(int64_t n) {
    (void)n;
    return 4 * 1024;
}

cgs_status cgs_loss_l1(const float* image, const float* target, int64_t n, float* grad, float* loss, void* ws,
                       size_t ws_bytes, void* stream) {
    if (n < 0 || !loss || !ws || (n > 0 && (!image || !target || !grad))) return CGS_EINVAL;
    if (ws_bytes < cgs_loss_l1_workspace_bytes(n)) return CGS_EWORKSPACE;
    int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    if (nb < 1) nb = 1;
    return hip_status(launch_l1(image, target, n, grad, loss, static_cast<float*>(ws), nb, static_cast<hipStream_t>(stream)));
}

namespace {
// Geometry of the loss batch; false on invalid sizes.
bool loss_views(int32_t n_views, const int32_t* hw, cgs::LossViews* lv, int64_t* n_pix) {
    if (n_views < 1 || n_views > CGS_MAX_VIEWS || !hw) return false;
    memset(lv, 0, sizeof(*lv));
    lv->n = n_views;
    int64_t p = 0, t = 0;
    for (int v = 0; v < n_views; ++v) {
        const int32_t H = hw[2 * v], W = hw[2 * v + 1];
        if (H <= 0 || W <= 0) return false;
        lv->H[v] = H;
        lv->W[v] = W;
        lv->tiles_x[v] = (W + cgs::kTile - 1) / cgs::kTile;
        lv->pix_off[v] = p;
        lv->tile_off[v] = t;
        p += (int64_t)H * W;
        t += (int64_t)lv->tiles_x[v] * ((H + cgs::kTile - 1) / cgs::kTile);
    }
    lv->tile_off[n_views] = t;
    *n_pix = p;
    return t < ((int64_t)1 << 31);
}
}  // namespace

size_t cgs_loss_recon_workspace_bytes(int32_t n_views, const int32_t* hw) {
    cgs::LossViews lv;
    int64_t P;
    if (!loss_views(n_views, hw, &lv, &P)) return 0;
    return align_up(36 * (size_t)P) + 16 * (size_t)lv.tile_off[n_views] + 256;
}

cgs_status cgs_loss_recon(const float* image, const float* target, int32_t n_views, const int32_t* hw,
                          float lambda_ssim, float* grad, float* loss, void* ws, size_t ws_bytes, void* stream) {
    cgs::LossViews lv;
    int64_t P;
    if (!loss_views(n_views, hw, &lv, &P)) return CGS_EINVAL;
    if (!(lambda_ssim >= 0.f && lambda_ssim <= 1.f)) return CGS_EINVAL;
    if (!image || !target || !grad || !loss || !ws) return CGS_EINVAL;
    if (ws_bytes < cgs_loss_recon_workspace_bytes(n_views, hw)) return CGS_EWORKSPACE;
    float* part = static_cast<float*>(ws);
    double* sums = reinterpret_cast<double*>(static_cast<char*>(ws) + align_up(36 * (size_t)P));
    return hip_status(cgs::launch_loss_recon(lv, image, target, lambda_ssim, grad, loss, part, sums,
                                             static_cast<hipStream_t>(stream)));
}

namespace {
// Host checks of a codebook under MH moves; fills the kernel arguments.
bool mh_args(const cgs_mh_codebook* cb, const cgs_mh* p, cgs::MhArgs* a) {
    if (!cb || !p || !cb->rows || !cb->d_rows) return false;
    if (cb->D < 1 || cb->D > 60 || cb->ld < cb->D || cb->K_max < 1 || cb->K_max >= ((int64_t)1 << 31)) return false;
    if (cb->n < 0 || cb->n >= ((int64_t)1 << 31) || (cb->n > 0 && !cb->idx)) return false;
    if (cb->mirror && cb->mirror_ld < cb->D) return false;
    if (p->n_proposals < 1 || !(p->lambda >= 0.f && p->lambda < 1e30f)) return false;
    if (!(p->eps_split > 0.f && p->eps_split < 1e30f) || !(p->eps_merge > 0.f && p->eps_merge < 1e30f)) return false;
    a->rows = cb->rows;
    a->ld = cb->ld;
    a->D = cb->D;
    a->K_max = cb->K_max;
    a->n = cb->n;
    a->d_rows = cb->d_rows;
    a->idx = cb->idx;
    a->mirror = cb->mirror;
    a->mirror_ld = cb->mirror_ld;
    a->lambda = p->lambda;
    a->inv_s2 = (float)(1.0 / ((double)p->eps_split * p->eps_split));
    a->inv_m2 = (float)(1.0 / ((double)p->eps_merge * p->eps_merge));
    a->eps_split = p->eps_split;
    a->B = p->n_proposals;
    a->seed = p->seed;
    a->step = p->step;
    return true;
}
}  // namespace

size_t cgs_mh_workspace_bytes(const cgs_mh_codebook* cb, int32_t n_proposals) {
    if (!cb || n_proposals < 1 || cb->D < 1 || cb->K_max < 1 || cb->n < 0) return 0;
    return cgs::mh_workspace(n_proposals, cb->D, cb->K_max, cb->n, nullptr, nullptr);
}

static cgs_status mh_run(const cgs_mh_codebook* cb, const cgs_mh* p, void* ws, size_t ws_bytes, void* stream,
                         bool split) {
    cgs::MhArgs a;
    if (!mh_args(cb, p, &a) || !ws) return CGS_EINVAL;
    cgs::MhWs w;
    const size_t need = cgs::mh_workspace(a.B, a.D, a.K_max, a.n, &w, static_cast<char*>(ws));
    if (ws_bytes < need) return CGS_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    return hip_status(split ? cgs::mh_split(a, w, st) : cgs::mh_merge(a, w, st));
}

cgs_status cgs_mh_split(const cgs_mh_codebook* cb, const cgs_mh* p, void* ws, size_t ws_bytes, void* stream) {
    return mh_run(cb, p, ws, ws_bytes, stream, true);
}

cgs_status cgs_mh_merge(const cgs_mh_codebook* cb, const cgs_mh* p, void* ws, size_t ws_bytes, void* stream) {
    return mh_run(cb, p, ws, ws_bytes, stream, false);
}

int32_t cgs_mh_transition(uint64_t seed, uint32_t step) { return cgs::mh_transition_host(seed, step); }

cgs_status cgs_sgld_normals(int64_t n, uint64_t index0, uint32_t tag, uint32_t step, uint64_t seed, float* z,
                            uint32_t* words, void* stream) {
    if (n < 0 || (n > 0 && !z)) return CGS_EINVAL;
    return hip_status(cgs::launch_normals(n, index0, tag, step, seed, z, words, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
