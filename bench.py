#!/usr/bin/env python3
"""Forward+backward rendered Mpixel/s of the codebook-indexed differentiable
Gaussian-splatting hot path on one MI355X.

A step is one pass of the whole path over one batch: preprocess (codebook
gather, projection, SH colour), tile binning (depth sort, emission, tile
sort), forward blend, L1 loss, backward blend, per-Gaussian chain rule and the
codebook-gradient reduction.  Inputs are seeded synthetic scenes resident in
HBM before the timed region.  The headline line measures the 4M-Gaussian,
BF16-codebook workload with its four 1957x1091 views in one batched call;
the plain-FP32 form (FP32 codebook, one call per view) and the 1M-Gaussian
workload are reported beside it in "forms".

Prints ONE JSON line.  --gpus N with N > 1 is refused: the benchmark
measures a single GPU.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2509_03775_amd import autotune, cgs, render, scenes as sc  # noqa: E402

METRIC = "fwd+bwd rendered Mpixel/s at 1M/4M Gaussians, BF16-batched vs plain FP32"
HEADLINE = "clusters4m_bf16_4x1957x1091"
VALU_PEAK = 256 * 4 * 16 * 2.4e9        # FP32 lane-operations/s, non-packed issue rate
FP32_PEAK = 157.3e12                    # MI355X FP32 vector peak (published; counts packed FMAs)
HBM_PEAK = 8.0e12                       # bytes/s
# The cost model of the blend stages: VALU operations per evaluated
# (pixel, Gaussian) pair, forward and backward, each priced against the
# published FP32 vector peak (the headline roofline and the combined
# per-stage roofline use these).
MODEL_OPS_FWD, MODEL_OPS_BWD = 20, 45
# Algorithmic FP32 operations per (pixel, Gaussian) pair (an FMA, an exp, a
# compare each count as one): alpha of a pair (2 sub, 5 for the quadratic
# form, exp, opacity product, 0.99 clamp, 1/255 test) = 11; a blended pair
# adds 8 in the forward (1-alpha, T product, T test, weight, 3 colour FMAs,
# count) and 30 in the backward (T recovery 2, weight 1, colour grads 3,
# alpha grad 7, background update 3, opacity grad 2, power grads 12).
OPS_ALPHA, OPS_FWD_BLEND, OPS_BWD_BLEND = 11, 8, 30
LAMBDA_SSIM = 0.2      # SSIM weight of the training-step form (Eq. 4)

# HBM bytes per launch of the blend kernels on the headline workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by what the same counter read for a 512 MiB torch.neg copy (FETCH
# 2.0, WRITE 1.0).  A figure holds only for the kernel sources and schedule it
# was taken on: the first 16 hex digits of the SHA-256 of those sources.
# The measured kernel's own source (its definition, from "template" to the
# closing brace, inside the named file) and the headers it includes.
KERNEL_SOURCES = {"k_blend_bwd": ("render_bwd.hip", ("render_common.h", "cgs_internal.h")),
                  "k_blend_fwd": ("render_fwd.hip", ("render_common.h", "cgs_internal.h"))}
MEASURED_TRAFFIC = {
    ("k_blend_bwd", HEADLINE, (1, 2, 0)): {"sources": "538e34f6b6ff3303", "read": 2653196947, "write": 729596960},
    ("k_blend_fwd", HEADLINE, (1, 2, 0)): {"sources": "9aa22205e39ba43c", "read": 1924572143, "write": 234870560},
}


def kernel_text(src: str, kernel: str) -> str:
    """The definition of `kernel` in a source file: from the template line
    (or the __global__ line) before its name to the first closing brace at
    column 0 after it."""
    at = src.index(" " + kernel + "(")
    start = src.rfind("\ntemplate", 0, at)
    glob = src.rfind("\n__global__", 0, at)
    start = max(start, glob) + 1
    end = src.index("\n}\n", at) + 3
    return src[start:end]


def sources_digest(kernel: str) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2509_03775_amd", "csrc")
    body_file, headers = KERNEL_SOURCES[kernel]
    with open(os.path.join(csrc, body_file)) as fh:
        h.update(kernel_text(fh.read(), kernel).encode())
    for f in headers:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, schedule) -> "int | None":
    """Counter-measured HBM bytes per launch, or None when no figure was
    taken for this kernel, workload and schedule or the kernel has changed
    since."""
    m = MEASURED_TRAFFIC.get((kernel, workload, tuple(schedule)))
    if m is None or m["sources"] != sources_digest(kernel):
        return None
    return m["read"] + m["write"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles created through the HIP runtime torch already loaded."""

    def __init__(self, n):
        self.lib = ctypes.CDLL("libamdhip64.so.7")
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.ev = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            rc = self.lib.hipEventCreate(ctypes.byref(h))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed ({rc})")
            self.ev[i] = h

    def slice(self, i, n):
        return ctypes.cast(ctypes.byref(self.ev, i * ctypes.sizeof(ctypes.c_void_p)), ctypes.POINTER(ctypes.c_void_p))

    def elapsed(self, i, j):
        out = ctypes.c_float()
        rc = self.lib.hipEventElapsedTime(ctypes.byref(out), self.ev[i], self.ev[j])
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return out.value


class Form:
    """One way to run a step: `batched` renders every view in one call; `plain`
    issues one call per view."""

    def __init__(self, wl: sc.Workload, batched: bool, capacity_slack=1.08, waves_per_block=1, tile_order=0,
                 train: bool = False, persistent: int = 0):
        self.wl = wl
        self.batched = batched
        self.train = train
        ds = [render.DeviceScene.from_host(s, bf16=wl.bf16) for s in wl.scenes]
        self.scenes = ds
        if batched:
            groups = [list(range(len(wl.cameras)))]
        else:
            groups = [[v] for v in range(len(wl.cameras))]
        self.renderers = []
        self.targets, self.grads, self.losses = [], [], []
        for gidx in groups:
            used = sorted(set(int(wl.view_scene[v]) for v in gidx))
            remap = {s: i for i, s in enumerate(used)}
            r = render.Renderer([ds[s] for s in used], [wl.cameras[v] for v in gidx],
                                [remap[int(wl.view_scene[v])] for v in gidx], waves_per_block=waves_per_block,
                                tile_order=tile_order, persistent=persistent)
            m = r.fit_capacity()
            r.set_capacity(int(m * capacity_slack) + 4096)
            r.fit_capacity()
            self.instances = getattr(self, "instances", 0) + m
            tgt = np.concatenate([wl.targets[v].reshape(-1, 3) for v in gidx], 0)
            self.targets.append(torch.from_numpy(tgt).cuda())
            self.grads.append(torch.empty_like(self.targets[-1]))
            self.losses.append(torch.zeros(1, device="cuda"))
            self.renderers.append(r)
        n = max(t.numel() for t in self.targets)
        self.loss_ws = torch.empty(cgs.loss_l1_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        self.n_pixels = wl.n_pixels
        if train:
            # Eq. 4 with the SSIM term and the SGLD update fused into the
            # backward; BF16 codebooks train an FP32 master (small steps keep
            # the scene, and so the instance count, essentially unchanged)
            self.masters = [None if s.cb.dtype == torch.float32 else s.cb.float() for s in ds]
            self.hw = [[(wl.cameras[v].height, wl.cameras[v].width) for v in gidx] for gidx in groups]
            self.recon_ws = [torch.empty(cgs.loss_recon_workspace_bytes(h), dtype=torch.uint8, device="cuda")
                             for h in self.hw]
            self.params = []
            for gidx in groups:
                used = sorted(set(int(wl.view_scene[v]) for v in gidx))
                self.params.append([render.sgld_params(ds[s], master_sr=self.masters[s]) for s in used])
            self.sgld = cgs.Sgld(1e-9, 1e-8, 1e-8, 1e-8, 2026, 0, 0)

    def step(self):
        if self.train:
            self.sgld.step += 1
            for i, (r, t, g, l) in enumerate(zip(self.renderers, self.targets, self.grads, self.losses)):
                img = r.forward()
                render.loss_recon(img, t, self.hw[i], LAMBDA_SSIM, g, l, self.recon_ws[i])
                r.backward_sgld(g, self.sgld, self.params[i])
            return
        for r, t, g, l in zip(self.renderers, self.targets, self.grads, self.losses):
            img = r.forward()
            render.loss_l1(img, t, g, l, self.loss_ws)
            r.backward(g)

    def time(self, steps, warmup, events: HipEvents = None):
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0 = self.renderers[0]
        e0.record()
        for k in range(steps):
            if events is not None:
                r0._sched.stage_events = events.slice(k * cgs.STAGE_EVENTS, cgs.STAGE_EVENTS)
            self.step()
        e1.record()
        torch.cuda.synchronize()
        if events is not None:
            r0._sched.stage_events = None
        return e0.elapsed_time(e1) / steps


def stage_times(ev: HipEvents, steps):
    names = [("preprocess", 0, 1), ("binning", 1, 2), ("blend_fwd", 2, 3), ("loss", 3, 4), ("blend_bwd", 4, 5),
             ("chain", 5, 6), ("codebook_reduce", 6, 7)]
    out = {}
    for name, a, b in names:
        out[name] = float(np.mean([ev.elapsed(k * cgs.STAGE_EVENTS + a, k * cgs.STAGE_EVENTS + b)
                                   for k in range(steps)]))
    return out


def step_distribution(ev: HipEvents, steps):
    """Median and 10th / 90th percentiles of the per-step GPU time, from the
    first to the last stage event of each timed step."""
    t = np.array([ev.elapsed(k * cgs.STAGE_EVENTS, k * cgs.STAGE_EVENTS + cgs.STAGE_EVENTS - 1)
                  for k in range(steps)])
    return {"median": float(np.median(t)), "p10": float(np.percentile(t, 10)), "p90": float(np.percentile(t, 90)),
            "of": "per-step GPU time, first to last stage event"}


def host_cpu():
    """The host CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cpus = sorted(os.sched_getaffinity(0))
    runs, a = [], None
    for i, c in enumerate(cpus):     # compact "0-15,32-47" form of the affinity mask
        if a is None:
            a = c
        if i + 1 == len(cpus) or cpus[i + 1] != c + 1:
            runs.append(f"{a}-{c}" if c > a else f"{a}")
            a = None
    return model, ",".join(runs), os.cpu_count()


def walked_instances(r: render.Renderer) -> int:
    """Instances the blends must read: per tile, list positions up to the
    largest n_last of its pixels (front-to-back termination)."""
    total = 0
    for v, cam in enumerate(r.cameras):
        nl = r.n_last[int(r.pix_off[v]):int(r.pix_off[v + 1])].view(cam.height, cam.width).to(torch.float32)
        th, tw = (cam.height + 15) // 16, (cam.width + 15) // 16
        pad = torch.zeros((th * 16, tw * 16), dtype=torch.float32, device=nl.device)
        pad[:cam.height, :cam.width] = nl
        total += int(torch.amax(pad.view(th, 16, tw, 16), dim=(1, 3)).to(torch.int64).sum().item())
    return total


def pair_counts(form: Form):
    """Pairs the backward evaluates (sum of n_last), pairs blended and
    instances walked."""
    e_eval = e_blend = walked = 0
    for r in form.renderers:
        r.forward()
        e_eval += int(r.n_last.to(torch.int64).sum().item())
        walked += walked_instances(r)
        nb = torch.zeros(r.n_pixels, dtype=torch.int32, device="cuda")
        r._sched.n_blend = nb.data_ptr()
        r.forward()
        torch.cuda.synchronize()
        r._sched.n_blend = None
        e_blend += int(nb.to(torch.int64).sum().item())
    return e_eval, e_blend, walked


def cpu_baseline(wl: sc.Workload, target_s: float, full_frames=("uniform4k_128px",)):
    """The FP64 oracle on a bounded sample of the same workload: forward, L1
    gradient and backward of randomly chosen 16x16 tiles of view 0."""
    import oracle
    cam, s = wl.cameras[0], wl.scenes[int(wl.view_scene[0])]
    P = wl.n_pixels
    rng = np.random.default_rng(7)
    tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16

    last = {}

    def run(ntiles):
        pick = rng.choice(tx * ty, size=ntiles, replace=False)
        pix = []
        for t in pick:
            x0, y0 = (t % tx) * 16, (t // tx) * 16
            yy, xx = np.mgrid[y0:min(y0 + 16, cam.height), x0:min(x0 + 16, cam.width)]
            pix.append(np.stack([xx.ravel(), yy.ravel()], 1))
        pix = np.concatenate(pix).astype(np.int32)
        t0 = time.perf_counter()
        o = oracle.render_view(s, cam, pix)
        t_fwd = time.perf_counter() - t0
        tgt = wl.targets[0][pix[:, 1], pix[:, 0]].astype(np.float64)
        g = np.sign(o["color"] - tgt) / (3.0 * P)
        g[o["ambiguous"]] = 0.0
        g32 = g.astype(np.float32)
        o2 = oracle.render_view(s, cam, pix, grad_color=g32.astype(np.float64))
        gcb = oracle.codebook_grad_reduce(o2["grad_rows"], s.idx, s.k)
        dt = time.perf_counter() - t0
        last.update(pix=pix, color=o["color"], ambiguous=o["ambiguous"], n_last=o["n_last"], g32=g32,
                    grad_means=o2["grad_means"], grad_cb=gcb)
        return dt, pix.shape[0], ntiles, t_fwd

    # each call projects the whole scene once (a fixed cost) and then
    # composites its tiles; grow the tile count until one call takes about
    # target_s, so the fixed cost is spread as it would be over a larger sample
    n_max = min(4096, tx * ty)
    n = min(2, n_max)
    dt, npix, ntiles, dt_fwd = run(n)
    while dt < 0.8 * target_s and n < n_max:
        n = int(min(n_max, max(2 * n, n * 0.9 * target_s / max(dt, 1e-3))))
        dt, npix, ntiles, dt_fwd = run(n)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    model, affinity, nproc = host_cpu()
    return {"value": npix / dt / 1e6, "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
            "cpu": model, "affinity": affinity, "nproc": nproc, "forward_value": npix / dt_fwd / 1e6,
            "full_frame": [cpu_full_frame(n) for n in full_frames],
            "sample": f"{ntiles} random 16x16 tiles ({npix} px) of view 0 of {wl.name}: FP64 forward, "
                      f"L1 gradient and backward incl. codebook reduction, {dt:.1f} s"}, last


def oracle_parity(form: "Form", sample: dict) -> dict:
    """The timed batched form against the FP64 oracle on the CPU baseline's
    sample (tiles of view 0): image error on non-ambiguous pixels, n_last
    mismatches, and per-block gradient errors of the L1 loss restricted to the
    sample (both sides given the same FP32 image gradient, zero elsewhere)."""
    r = form.renderers[0]
    cam = r.cameras[0]
    pix = sample["pix"]
    lin = pix[:, 1].astype(np.int64) * cam.width + pix[:, 0]
    r.forward()
    torch.cuda.synchronize()
    img = r.image[:cam.width * cam.height].cpu().numpy().astype(np.float64)[lin]
    nl = r.n_last[:cam.width * cam.height].cpu().numpy()[lin]
    ok = ~sample["ambiguous"]
    gimg = torch.zeros((r.n_pixels, 3), dtype=torch.float32)
    gimg[torch.from_numpy(lin)] = torch.from_numpy(sample["g32"])
    gm, gcb = r.backward(gimg.cuda())
    torch.cuda.synchronize()
    gcb, gm = gcb[0].cpu().numpy().astype(np.float64), gm[0].cpu().numpy().astype(np.float64)
    ocb, om = sample["grad_cb"], sample["grad_means"]

    def rel(a, b):
        nb = np.linalg.norm(b)
        return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))
    return {"pixels": int(len(lin)), "ambiguous": int((~ok).sum()),
            "image_max_abs": float(np.abs(img[ok] - sample["color"][ok]).max()),
            "n_last_mismatches": int((nl[ok] != sample["n_last"][ok]).sum()),
            "grad_rel_l2": {"means": rel(gm, om), **{k: rel(gcb[:, sl], ocb[:, sl]) for k, sl in GRAD_BLOCKS.items()}},
            "of": "view 0, the CPU baseline's sampled tiles"}


def cpu_full_frame(name: str):
    """The FP64 oracle on every pixel of a small workload's first view:
    forward alone, then forward, L1 gradient, backward and codebook
    reduction."""
    import oracle
    wl = sc.make_workload(name)
    s, cam = wl.scenes[int(wl.view_scene[0])], wl.cameras[0]
    P = cam.width * cam.height
    log(f"[bench] oracle full frame of {name}: forward")
    t0 = time.perf_counter()
    o = oracle.render_view(s, cam)
    t_fwd = time.perf_counter() - t0
    log(f"[bench] oracle full frame of {name}: forward {t_fwd:.1f} s, now L1 gradient and backward")
    tgt = wl.targets[0].reshape(-1, 3).astype(np.float64)
    g = np.sign(o["color"] - tgt) / (3.0 * P)
    o2 = oracle.render_view(s, cam, grad_color=g)
    oracle.codebook_grad_reduce(o2["grad_rows"], s.idx, s.k)
    t_all = time.perf_counter() - t0
    log(f"[bench] oracle full frame of {name}: forward + backward {t_all:.1f} s")
    return {"workload": name, "pixels": P, "forward": P / t_fwd / 1e6, "forward_backward": P / t_all / 1e6,
            "unit": "Mpixel/s"}


def blend_roofline(stage, ms, e_eval, e_blend, workload, schedule):
    """Roofline of one blend launch.  Headline figures: the cost model's VALU
    operations per evaluated pair (MODEL_OPS_*) times the evaluated pairs of
    the launch, divided by its measured duration, against the published FP32
    vector peak.  issue_model: the finer count (11 per evaluated pair plus 8
    or 30 per blended pair) against the non-packed issue rate."""
    kernel = "k_blend_bwd" if stage == "blend_bwd" else "k_blend_fwd"
    per_pair = MODEL_OPS_BWD if stage == "blend_bwd" else MODEL_OPS_FWD
    ops = per_pair * e_eval
    ach = ops / (ms * 1e-3)
    fine = OPS_ALPHA * e_eval + (OPS_BWD_BLEND if stage == "blend_bwd" else OPS_FWD_BLEND) * e_blend
    return {"bound": "alu", "achieved": ach / 1e12, "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / FP32_PEAK, "traffic": measured_traffic(kernel, workload, schedule), "kernel": kernel,
            "model": f"{per_pair} VALU ops per evaluated pair x {e_eval} evaluated pairs per launch",
            "ops_per_launch": ops, "launch_ms": ms,
            "issue_model": {"ops_per_launch": fine, "achieved": fine / (ms * 1e-3) / 1e12,
                            "peak": VALU_PEAK / 1e12, "unit": "T lane-ops/s",
                            "frac": fine / (ms * 1e-3) / VALU_PEAK}}


def combined_roofline(stages_ms: dict, sb: dict, e_eval: int, step_ms: float) -> dict:
    """Sum over stages of max(bytes / HBM peak, VALU ops / FP32 peak) against
    the measured step: the blends priced by the cost model's operations per
    evaluated pair, every other stage by its algorithmic bytes."""
    ops = {"blend_fwd": MODEL_OPS_FWD * e_eval, "blend_bwd": MODEL_OPS_BWD * e_eval}
    per = {}
    for k in stages_ms:
        t_b = sb.get(k, 0) / HBM_PEAK
        t_o = ops.get(k, 0) / FP32_PEAK
        per[k] = {"roof_ms": 1e3 * max(t_b, t_o), "bound": "alu" if t_o > t_b else "hbm",
                  "measured_ms": stages_ms[k], "frac": 1e3 * max(t_b, t_o) / stages_ms[k] if stages_ms[k] else None}
    t_roof = sum(v["roof_ms"] for v in per.values())
    return {"roof_ms": t_roof, "step_ms": step_ms, "frac": t_roof / step_ms, "stages": per}


def depth_sort_passes(wl: sc.Workload) -> int:
    """Passes of 9-bit digits the records' depth sort takes: its keys are the
    bit patterns of the FP32 camera depths in front of the near plane, sorted
    relative to the least of them (host estimate; the device decides)."""
    lo, hi = None, None
    for v, cam in enumerate(wl.cameras):
        m = wl.scenes[int(wl.view_scene[v])].means
        z = (m @ cam.Rt[2, :3].astype(np.float32) + np.float32(cam.Rt[2, 3])).astype(np.float32)
        z = z[z > np.float32(0.2)]
        if z.size == 0:
            continue
        k = z.view(np.uint32)
        lo = int(k.min()) if lo is None else min(lo, int(k.min()))
        hi = int(k.max()) if hi is None else max(hi, int(k.max()))
    bits = max(1, (hi - lo).bit_length()) if lo is not None else 1
    return (bits + 8) // 9


def step_bytes(wl: sc.Workload, n_inst: int, walked: int) -> dict:
    """Algorithmic HBM bytes of one step, per stage: what the method must
    read and write once (codebook rows counted once per unique row; a radix
    pass reads and writes each item once, plus one key read per sort for the
    digit counts of all its passes).  Binning: the depth sort (key, record
    and packed rectangle, 12 B per record each way per pass, as many 9-bit
    passes as the live depth range needs), the offsets scan (8 B per record),
    the emission (20 B in per record, tile key + record out per instance,
    the key in 2 B when the batch has at most 65536 tiles), the slot-offset
    scan and the tile sort.  The blends read only the walked instances W
    (positions before the tile's termination): a 4 B record id plus the
    record's 36 B of blend data each; the backward adds the record's tile
    rectangle and slot offset (12 B) and writes a 36 B gradient slot.  The
    chain rule reads those slots back (with each record's depth key and its
    rectangle, one packed word when every view is below 256 tiles per side,
    else 8 B and a 4 B tile count), the Gaussians in row order (8 B of
    sorted row and id each) and writes dL/dmean, each wavefront's two partial
    rows and the codebook gradient; the reduction stage is the row sort and
    the merge of the partial rows."""
    N = sum(s.n for s in wl.scenes)
    Rrec = sum(wl.scenes[int(v)].n for v in wl.view_scene)
    K = sum(s.k for s in wl.scenes)
    RW = wl.scenes[0].r
    b = 2 if wl.bf16 else 4
    P = wl.n_pixels
    M = n_inst
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in wl.cameras)
    tile_passes = (max(1, (tiles - 1).bit_length()) + 7) // 8
    key_b = 2 if tiles <= 65536 else 4
    row_passes = (max(1, (K - 1).bit_length()) + 7) // 8
    partials = 2 * ((N + 63) // 64) * 4 * RW
    packed = all((c.width + 15) // 16 < 256 and (c.height + 15) // 16 < 256 for c in wl.cameras)
    rect_b = 4 if packed else 12
    out = {
        "preprocess": N * 16 + K * RW * b + Rrec * 52,
        "binning": (depth_sort_passes(wl) * 24 + 4 + 8 + 20 + 8) * Rrec
        + ((key_b + 4) + key_b + tile_passes * 2 * (key_b + 4)) * M,
        "blend_fwd": walked * 40 + P * 20,
        "loss": P * 36,
        "blend_bwd": walked * (40 + 12 + 36) + P * 24 + tiles * 8,
        "chain": N * 16 + K * RW * b + Rrec * (8 + rect_b) + walked * 36 + tiles * 8 + N * 8 + N * 12 + partials + K * 4 * RW,
        "codebook_reduce": N * 8 + row_passes * 16 * N + 4 * N + partials + K * 8,
    }
    out["total"] = sum(out.values())
    return out


GRAD_BLOCKS = {"ls": slice(0, 3), "q": slice(3, 7), "logit": slice(7, 8), "sh_dc": slice(8, 11),
               "sh_rest": slice(11, None)}


def _weighted_grads(form: "Form"):
    """Codebook and mean gradients of a form, each call's share weighted by
    its pixels over the batch's: the loss of every call is a mean over that
    call's pixels, so this puts a one-call-per-view form on the same
    normalisation (mean over the whole batch) as the batched form."""
    gc = gm = 0
    for r in form.renderers:
        w = r.n_pixels / form.n_pixels
        gc = gc + w * r.grad_cb[0].double()
        gm = gm + w * r.grad_means[0].double()
    return gc, gm


def compare_forms(a: "Form", b: "Form"):
    """Image and gradient difference between two forms of the same scene
    (BF16 vs FP32 codebook storage: the quantisation effect), after one step
    of each; gradients per parameter block, relative L2 against b."""
    ia = torch.cat([r.image for r in a.renderers]).double()
    ib = torch.cat([r.image for r in b.renderers]).double()
    ga, ma = _weighted_grads(a)
    gb, mb = _weighted_grads(b)

    def rel(x, y):
        return float(torch.linalg.norm(x - y) / torch.linalg.norm(y))
    out = {"image_max_abs": float((ia - ib).abs().max()), "image_mean_abs": float((ia - ib).abs().mean()),
           "codebook_grad_rel_l2": rel(ga, gb), "means_grad_rel_l2": rel(ma, mb)}
    out["codebook_grad_rel_l2_by_block"] = {k: rel(ga[:, sl], gb[:, sl]) for k, sl in GRAD_BLOCKS.items()}
    return out


def check_form(form: "Form") -> dict:
    """Device-side conditions of the form's last step: every call had the
    instance capacity it needed, and no radix-sort wait reached its bound
    (either would make the timed step do less than the full work)."""
    torch.cuda.synchronize()
    info = [r.d_info.cpu().numpy() for r in form.renderers]
    ok = all(int(i[0]) == cgs.CGS_OK for i in info)
    stalls = int(cgs.load().cgs_sort_stalls())
    if not ok or stalls != 0:
        raise RuntimeError(f"bench: a timed step was incomplete (d_info {[list(map(int, i)) for i in info]}, "
                           f"sort stalls {stalls})")
    return {"capacity_ok": ok, "sort_stalls": stalls}


def uncompressed_workload(wl: sc.Workload) -> sc.Workload:
    """Same Gaussians with one codebook row per Gaussian (K = N, identity
    indices): the uncompressed per-Gaussian-parameter baseline."""
    scenes = []
    for s in wl.scenes:
        cb = np.ascontiguousarray(s.cb[s.idx])
        bits = None if s.cb_bf16 is None else np.ascontiguousarray(s.cb_bf16[s.idx])
        scenes.append(sc.Scene(s.means, np.arange(s.n, dtype=np.int32), cb, s.sh_degree, bits))
    return sc.Workload(wl.name + ":uncompressed", scenes, wl.cameras, wl.view_scene, wl.targets, wl.bf16)


def time_moves(wl: sc.Workload, n_proposals: int = 4096, reps: int = 10) -> dict:
    """Split and merge moves on the workload's first codebook (FP32 master
    with room for 2K rows, BF16 copy refreshed): mean ms per call over `reps`
    calls of each, the state carried from call to call."""
    s = wl.scenes[0]
    K, R = s.cb.shape
    rows = torch.zeros((2 * K, R), dtype=torch.float32, device="cuda")
    rows[:K] = torch.from_numpy(np.ascontiguousarray(s.cb)).cuda()
    mirror = torch.zeros((2 * K, R), dtype=torch.int16, device="cuda")
    idx = torch.from_numpy(np.ascontiguousarray(s.idx)).cuda()
    mv = render.CodebookMoves(rows, K, idx, mirror=mirror, n_proposals=n_proposals)
    out = {"gaussians": s.n, "rows": int(K), "row_width": int(R), "proposals": n_proposals}
    for kind in ("split", "merge"):
        fn = mv.split if kind == "split" else mv.merge
        fn(mv.params(2.3, 0.1, 0.05, 1, 0))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(reps):
            fn(mv.params(2.3, 0.1, 0.05, 1, 1 + k))
        e1.record()
        torch.cuda.synchronize()
        out[f"{kind}_ms"] = e0.elapsed_time(e1) / reps
    out["live_rows_after"] = mv.live_rows()
    return out


def time_graph(form: "Form", steps: int) -> float:
    """One step captured in a HIP graph, replayed `steps` times."""
    form.step()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        form.step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        form.step()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--extra-forms", default="train,mh,fp32_plain,1m,uncompressed,uneven16,graph",
                    help="comma list of: fp32_plain, 1m, uncompressed, uneven16, graph; or none")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-full-frame", default="uniform4k_128px,clusters200k_800px",
                    help="comma list of workloads whose first view the oracle renders in full "
                         "(clusters200k_800px takes about 16 s on 16 cores)")
    ap.add_argument("--schedule", default="auto",
                    help="blend schedule 'W,O' (waves per workgroup, tile order) or 'auto' to time the candidates")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a device-to-device copy of this many MiB (a kernel of known traffic "
                         "for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; multi-GPU use would shard the views)", file=sys.stderr)
        sys.exit(2)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cgs.load()
    torch.cuda.set_device(0)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.arange(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.copy_calibration_mib} MiB read + {args.copy_calibration_mib} MiB written")
        del src, dst
    log(f"[bench] generating {args.workload}")
    wl = sc.make_workload(args.workload)
    head = Form(wl, batched=True)
    tuned = {}
    if args.schedule == "auto":
        log("[bench] timing the blend schedule candidates")
        head.step()
        sched, tuned = autotune.tune(head.renderers[0], head.grads[0], reps=3, use_cache=False)
    else:
        sched = tuple(int(x) for x in args.schedule.split(","))
        sched = sched + (0,) * (3 - len(sched))
        head.renderers[0].set_schedule(*sched)
    log(f"[bench] schedule waves_per_block={sched[0]} tile_order={sched[1]} persistent={sched[2]}")
    ev = HipEvents(args.steps * cgs.STAGE_EVENTS)
    log(f"[bench] timing {args.workload} batched: {args.steps} steps after {args.warmup} warmup")
    ms = head.time(args.steps, args.warmup, ev)
    stages = stage_times(ev, args.steps)
    step_dist = step_distribution(ev, args.steps)
    value = wl.n_pixels / (ms * 1e-3) / 1e6
    checks = {"batched": check_form(head)}
    e_eval, e_blend, walked = pair_counts(head)
    dom = max(("blend_fwd", "blend_bwd"), key=lambda k: stages[k])
    roof = blend_roofline(dom, stages[dom], e_eval, e_blend, args.workload, sched)
    forms = {f"{'bf16' if wl.bf16 else 'fp32'}_batched:{args.workload}": value}
    n_inst = head.instances
    extras = [x for x in args.extra_forms.split(",") if x and x != "none"]
    extra_info = {}
    nsteps = max(3, args.steps // 2)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s) and the oracle check of its sample")
        cpu, sample = cpu_baseline(wl, args.cpu_seconds,
                                   tuple(x for x in args.cpu_full_frame.split(",") if x))
        extra_info["oracle_parity"] = oracle_parity(head, sample)
        del sample
    if "graph" in extras:
        log("[bench] timing the batched step as HIP graph replays")
        extra_info["graph_ms_per_step"] = time_graph(head, nsteps)
        checks["graph"] = check_form(head)
        forms[f"{'bf16' if wl.bf16 else 'fp32'}_batched_graph:{args.workload}"] = \
            wl.n_pixels / (extra_info["graph_ms_per_step"] * 1e-3) / 1e6
    if "fp32_plain" in extras:
        log(f"[bench] timing {args.workload} plain fp32")
        wl32 = sc.make_workload(args.workload, bf16=False)
        f = Form(wl32, batched=False)      # plain: default schedule, one call per view
        forms[f"fp32_plain:{args.workload}"] = wl32.n_pixels / (f.time(nsteps, 2) * 1e-3) / 1e6
        checks["fp32_plain"] = check_form(f)
        if wl.bf16:
            head.step()
            torch.cuda.synchronize()
            extra_info["bf16_vs_fp32_codebook"] = compare_forms(head, f)
        del f, wl32
        torch.cuda.empty_cache()
    if "train" in extras:
        log(f"[bench] timing {args.workload} training step: SSIM loss + fused SGLD update")
        f = Form(wl, batched=True, waves_per_block=sched[0], tile_order=sched[1], train=True, persistent=sched[2])
        ev2 = HipEvents(nsteps * cgs.STAGE_EVENTS)
        ms_t = f.time(nsteps, 2, ev2)
        checks["train"] = check_form(f)
        st2 = stage_times(ev2, nsteps)
        forms[f"{'bf16' if wl.bf16 else 'fp32'}_batched_train_ssim_sgld:{args.workload}"] = wl.n_pixels / (ms_t * 1e-3) / 1e6
        extra_info["train_step"] = {
            "ms_per_step": ms_t, "lambda_ssim": LAMBDA_SSIM, "stages_ms": st2,
            "loss_ssim_minus_l1_ms": st2["loss"] - stages["loss"],
            "sgld_epilogues_ms": (st2["chain"] + st2["codebook_reduce"]) - (stages["chain"] + stages["codebook_reduce"])}
        del f, ev2
        torch.cuda.empty_cache()
    if "mh" in extras:
        log("[bench] timing the split and merge moves")
        extra_info["mh_moves"] = time_moves(wl)
    if "uncompressed" in extras:
        log(f"[bench] timing {args.workload} uncompressed (K = N)")
        wu = uncompressed_workload(wl)
        f = Form(wu, batched=True, waves_per_block=sched[0], tile_order=sched[1], persistent=sched[2])
        ms_u = f.time(nsteps, 2)
        checks["uncompressed"] = check_form(f)
        forms[f"{'bf16' if wl.bf16 else 'fp32'}_batched_uncompressed:{args.workload}"] = wl.n_pixels / (ms_u * 1e-3) / 1e6
        extra_info["codebook_speedup_vs_uncompressed"] = ms_u / ms
        del f, wu
        torch.cuda.empty_cache()
    del head
    torch.cuda.empty_cache()
    if "1m" in extras:
        name = "clusters1m_1600x1064"
        for bf in (True, False):
            log(f"[bench] timing {name} {'bf16 batched' if bf else 'fp32 plain'}")
            w1 = sc.make_workload(name, bf16=bf)
            f = Form(w1, batched=bf, waves_per_block=sched[0] if bf else 1, tile_order=sched[1] if bf else 0,
                     persistent=sched[2] if bf else 0)
            forms[f"{'bf16_batched' if bf else 'fp32_plain'}:{name}"] = \
                w1.n_pixels / (f.time(nsteps, 2) * 1e-3) / 1e6
            checks[f"{'bf16_batched' if bf else 'fp32_plain'}:{name}"] = check_form(f)
            del f
            torch.cuda.empty_cache()
    if "uneven16" in extras:
        # 16 uneven scenes: plain FP32 (16 sequential calls, default schedule)
        # against one batched BF16 call per stage, graph-replayed, with the
        # schedule tuned on this batch; the grid launch and the persistent
        # tile queue are both timed under replay and the faster is the form.
        name = "uneven16_512px"
        log(f"[bench] timing {name} fp32 plain (16 calls)")
        w5 = sc.make_workload(name, bf16=False)
        f = Form(w5, batched=False)
        forms[f"fp32_plain:{name}"] = w5.n_pixels / (f.time(nsteps, 2) * 1e-3) / 1e6
        checks[f"fp32_plain:{name}"] = check_form(f)
        del f
        torch.cuda.empty_cache()
        w5 = sc.make_workload(name, bf16=True)
        f = Form(w5, batched=True)
        f.step()
        s5, tuned5 = autotune.tune(f.renderers[0], f.grads[0], reps=3, use_cache=False)
        grid = min((c for c in autotune.CANDIDATES if c[2] == 0), key=lambda c: tuned5[",".join(map(str, c))])
        pers = min((c for c in autotune.CANDIDATES if c[2] == 1), key=lambda c: tuned5[",".join(map(str, c))])
        by = {}
        for label, c in (("grid", grid), ("persistent", pers)):
            log(f"[bench] timing {name} bf16 batched graph, {label} schedule {c}")
            f.renderers[0].set_schedule(*c)
            by[label] = {"schedule": list(c), "ms": time_graph(f, nsteps)}
            checks[f"bf16_batched_graph_{label}:{name}"] = check_form(f)
        best = min(by, key=lambda k: by[k]["ms"])
        forms[f"bf16_batched_graph:{name}"] = w5.n_pixels / (by[best]["ms"] * 1e-3) / 1e6
        extra_info["uneven16_batched"] = {"tuned_ms": tuned5, "graph_ms": by, "kept": best,
                                          "grid_mpix_s": w5.n_pixels / (by["grid"]["ms"] * 1e-3) / 1e6,
                                          "persistent_mpix_s": w5.n_pixels / (by["persistent"]["ms"] * 1e-3) / 1e6}
        del f
        torch.cuda.empty_cache()
    cam = wl.cameras[0]
    sb = step_bytes(wl, n_inst, walked)
    out = {
        "metric": METRIC, "value": value, "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "form": "batched", "codebook_storage": "bf16" if wl.bf16 else "f32",
                   "gaussians": int(sum(s.n for s in wl.scenes)), "codebook_rows": int(wl.scenes[0].k),
                   "sh_degree": int(wl.scenes[0].sh_degree), "views": len(wl.cameras),
                   "resolution": f"{cam.width}x{cam.height}", "pixels": int(wl.n_pixels)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
        "stages_ms": stages,
        "step_ms_dist": step_dist,
        "hbm_roofline_step": {"algorithmic_bytes": sb["total"], "bytes_by_stage": sb,
                              "frac": sb["total"] / HBM_PEAK / (ms * 1e-3)},
        "combined_roofline_step": combined_roofline(stages, sb, e_eval, ms),
        "checks": checks,
        "extra": extra_info,
        "pairs": {"evaluated": e_eval, "blended": e_blend, "instances": n_inst, "walked_instances": walked},
        "schedule": {"waves_per_block": sched[0], "tile_order": sched[1], "persistent": sched[2],
                     "candidates_ms": tuned},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
