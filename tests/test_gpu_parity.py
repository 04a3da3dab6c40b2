"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Integer work (depth keys, tile rectangles, binning, n_last) must match bit for
bit; images within 1e-4 max-abs on non-ambiguous pixels; gradients within
1e-3 relative L2 per parameter block."""
import zlib

import numpy as np
import pytest
import torch

import oracle
from paper_2509_03775_amd import cgs, render, scenes as sc
from harness import (BLOCKS, GRAD_TOL, IMAGE_TOL, compare_view, full_pixels, grad_error_stats, grad_errors,
                     oracle_grad_image, oracle_render, oracle_scene_grads, random_tiles, record, rel_l2, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cgs.load()
    yield
    torch.cuda.synchronize()


def small_workload(kind: str) -> sc.Workload:
    """Small seeded workloads spanning several tiles with ragged edges."""
    if kind == "uniform4k_128px":
        return sc.make_workload("uniform4k_128px")
    rng = np.random.default_rng({"clusters20k_d3": 71, "clusters20k_d3_bf16": 72, "views3": 73,
                                 "scenes3": 74, "ragged_d1": 75, "wide258": 76, "degenerate": 77, "mixed_views": 78}[kind])
    if kind in ("clusters20k_d3", "clusters20k_d3_bf16"):
        bf = kind.endswith("bf16")
        s = sc.make_scene(rng, 20000, 512, 3, sc.screen_matched_mu(200), clusters=True, bf16=bf)
        cams = [sc.pinhole(200, 152, (0.4, -0.3, -3.0))]
        return sc.Workload(kind, [s], cams, np.array([0], np.int32),
                           [rng.uniform(0, 1, (152, 200, 3)).astype(np.float32)], bf)
    if kind == "views3":
        s = sc.make_scene(rng, 8000, 300, 2, sc.screen_matched_mu(96), clusters=True)
        cams = [sc.pinhole(96, 80, (3.0 * np.sin(a), 0.2, -3.0 * np.cos(a))) for a in (0.0, 2.0, 4.0)]
        return sc.Workload(kind, [s], cams, np.array([0, 0, 0], np.int32),
                           [rng.uniform(0, 1, (80, 96, 3)).astype(np.float32) for _ in cams], False)
    if kind == "scenes3":
        ss = [sc.make_scene(rng, n, k, 3, sc.screen_matched_mu(64), clusters=True) for n, k in
              ((3000, 64), (500, 200), (7000, 1000))]
        cams = [sc.pinhole(64, 48, (0.0, 0.0, -3.0)), sc.pinhole(40, 72, (0.5, 0.0, -3.0)),
                sc.pinhole(64, 64, (0.0, 0.5, -3.0))]
        return sc.Workload(kind, ss, cams, np.array([2, 0, 1], np.int32),
                           [rng.uniform(0, 1, (c.height, c.width, 3)).astype(np.float32) for c in cams], False)
    if kind == "mixed_views":
        # scenes with 2, 3, 0 and 1 views, the views interleaved across the
        # scenes, and a last scene of 130 Gaussians (a ragged last wavefront)
        ss = [sc.make_scene(rng, n, k, 2, sc.screen_matched_mu(64), clusters=True) for n, k in
              ((2500, 64), (4000, 200), (900, 100), (130, 16))]
        cams = [sc.pinhole(64, 48, (3.0 * np.sin(a), 0.1, -3.0 * np.cos(a))) for a in (0.0, 0.7, 1.4, 2.1, 2.8)]
        cams.append(sc.pinhole(72, 40, (0.2, -0.2, -3.0)))
        return sc.Workload(kind, ss, cams, np.array([1, 0, 1, 3, 1, 0], np.int32),
                           [rng.uniform(0, 1, (c.height, c.width, 3)).astype(np.float32) for c in cams], False)
    if kind == "ragged_d1":
        s = sc.make_scene(rng, 3000, 100, 1, -3.2, clusters=False)
        cams = [sc.pinhole(77, 45, (0.1, 0.1, -2.5))]
        return sc.Workload(kind, [s], cams, np.array([0], np.int32),
                           [rng.uniform(0, 1, (45, 77, 3)).astype(np.float32)], False)
    if kind == "wide258":
        # 258 tiles across: the depth sort gathers tile rectangles instead of
        # carrying them packed in one word (fewer than 256 tiles per side)
        s = sc.make_scene(rng, 20000, 256, 1, sc.screen_matched_mu(600), clusters=False)
        cams = [sc.pinhole(4120, 72, (0.0, 0.0, -3.0))]
        return sc.Workload(kind, [s], cams, np.array([0], np.int32),
                           [rng.uniform(0, 1, (72, 4120, 3)).astype(np.float32)], False)
    if kind == "degenerate":
        # Gaussians that cover the whole 20 x 15-tile frame (records with
        # ~300 tile slots), large ones centred outside the clamped frustum
        # (the Jacobian's clamp branches), and Gaussians behind the camera
        # or far off screen (culled)
        s = sc.make_scene(rng, 3000, 128, 3, sc.screen_matched_mu(320), clusters=True)
        cb, means, idx = s.cb.copy(), s.means.copy(), s.idx.copy()
        cb[0, 0:3] = np.log(0.8)        # row 0: 3 sigma ~ 220 px at depth 3
        cb[0, 7] = -1.5                 # low opacity: the scene behind still blends
        idx[:9] = 0
        means[:6] = rng.uniform(-0.3, 0.3, (6, 3))
        means[6:9] = np.array([[3.0, 0.2, 0.0], [-3.2, -0.1, 0.3], [0.1, 2.6, 0.0]])
        means[9:59, 2] = -4.5           # behind the camera at z = -3
        means[59:109, 0] = 40.0         # far to the side
        s = sc.Scene(means, idx, cb, 3)
        cams = [sc.pinhole(320, 240, (0.0, 0.0, -3.0))]
        return sc.Workload(kind, [s], cams, np.array([0], np.int32),
                           [rng.uniform(0, 1, (240, 320, 3)).astype(np.float32)], False)
    raise KeyError(kind)


def gpu_renderer(wl: sc.Workload, **kw) -> render.Renderer:
    ds = [render.DeviceScene.from_host(s, bf16=wl.bf16) for s in wl.scenes]
    r = render.Renderer(ds, wl.cameras, wl.view_scene, **kw)
    r.fit_capacity()
    return r


SMALL = ["uniform4k_128px", "clusters20k_d3", "clusters20k_d3_bf16", "views3", "scenes3", "mixed_views", "ragged_d1",
         "wide258", "degenerate"]


@pytest.mark.parametrize("kind", SMALL)
def test_skeleton_bit_exact(kind):
    wl = small_workload(kind)
    say(f"[skeleton] {kind}")
    r = gpu_renderer(wl)
    torch.cuda.synchronize()
    lay = r.layout()
    ws = r.ws.cpu().numpy()
    R = lay.n_records
    key = ws[lay.depth_key:lay.depth_key + 4 * R].view(np.uint32)
    tr = ws[lay.records:lay.records + 48 * R].view(np.uint32).reshape(R, 12)[:, 9:11]   # the record's rectangle words
    off = 0
    for v, cam in enumerate(wl.cameras):
        s = wl.scenes[int(wl.view_scene[v])]
        rows = oracle.decode_rows(s)
        okey, otr, okept = oracle.keyspec(s.means, rows[:, :7], cam)
        gk = key[off:off + s.n]
        gt = tr[off:off + s.n]
        gkept = gk != 0x7F800000
        np.testing.assert_array_equal(gkept, okept)
        np.testing.assert_array_equal(gk[okept], okey[okept])
        g4 = np.stack([gt[:, 0] & 0xFFFF, gt[:, 0] >> 16, gt[:, 1] & 0xFFFF, gt[:, 1] >> 16], 1)
        np.testing.assert_array_equal(g4[okept], otr[okept].astype(np.uint32))
        off += s.n


@pytest.mark.parametrize("kind", SMALL)
def test_forward_full_frame(kind):
    wl = small_workload(kind)
    say(f"[forward] {kind}")
    r = gpu_renderer(wl)
    r.forward()
    torch.cuda.synchronize()
    img, T, nl = r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy()
    pix = [full_pixels(c) for c in wl.cameras]
    outs = oracle_render(wl, pix)
    views = []
    for v, cam in enumerate(wl.cameras):
        a, b = r.pix_off[v], r.pix_off[v + 1]
        ec, et, mism, namb = compare_view(img[a:b], T[a:b], nl[a:b], cam, pix[v], outs[v])
        say(f"  view {v}: colour err {ec:.2e} T err {et:.2e} n_last mismatches {mism} ambiguous {namb}/{len(pix[v])}")
        views.append({"image_max_abs": ec, "T_max_abs": et, "ambiguous": namb, "pixels": int(len(pix[v]))})
        assert ec <= IMAGE_TOL and et <= IMAGE_TOL and mism == 0
        assert namb <= 0.01 * len(pix[v])
    record(kind + ":forward", views=views)


@pytest.mark.parametrize("kind", SMALL)
def test_backward_full_frame(kind):
    wl = small_workload(kind)
    say(f"[backward] {kind}")
    r = gpu_renderer(wl)
    pix = [full_pixels(c) for c in wl.cameras]
    base = oracle_render(wl, pix)
    gcols, gfull = oracle_grad_image(wl, pix, base)
    outs = oracle_render(wl, pix, gcols)
    ogm, ogcb = oracle_scene_grads(wl, outs)
    r.forward()
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    scenes_rec = []
    for i in range(len(wl.scenes)):
        errs = grad_errors(gm[i].cpu().numpy(), gcb[i].cpu().numpy(), ogm[i], ogcb[i])
        scenes_rec.append(grad_error_stats(gm[i].cpu().numpy(), gcb[i].cpu().numpy(), ogm[i], ogcb[i]))
        say(f"  scene {i}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        for k, e in errs.items():
            assert e <= GRAD_TOL, (k, e)
    record(kind + ":backward", grads=scenes_rec)


def test_determinism():
    wl = small_workload("clusters20k_d3")
    say("[determinism] clusters20k_d3")
    r = gpu_renderer(wl)
    g = torch.from_numpy(np.random.default_rng(5).standard_normal((r.n_pixels, 3)).astype(np.float32) * 1e-5).cuda()
    outs = []
    for _ in range(2):
        r.forward()
        _, gcb = r.backward(g)
        torch.cuda.synchronize()
        outs.append((r.image.cpu().numpy().copy(), gcb[0].cpu().numpy().copy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("kind", ["scenes3", "views3", "mixed_views"])
def test_schedule_invariance(kind):
    """Waves per workgroup, tile order and the persistent tile queue change
    only the issue order: every output (image, T, n_last, every gradient) is
    bitwise the same.  A persistent renderer also runs the step twice more,
    the second time with two backwards after one forward, which needs each
    launch to leave its tile queue reset for the next."""
    wl = small_workload(kind)
    g = torch.from_numpy(np.random.default_rng(6).standard_normal((sum(c.width * c.height for c in wl.cameras), 3))
                         .astype(np.float32) * 1e-5).cuda()
    ref = None
    for wpb, order, pers in ((1, 0, 0), (2, 1, 0), (4, 2, 0), (1, 2, 0), (2, 2, 0), (1, 0, 1), (1, 2, 1)):
        say(f"[schedule] {kind} waves_per_block={wpb} tile_order={order} persistent={pers}")
        r = gpu_renderer(wl, waves_per_block=wpb, tile_order=order, persistent=pers)
        for rep in range(3 if pers else 1):
            r.forward()
            if rep == 2:
                r.backward(g)
            _, gcb = r.backward(g)
            torch.cuda.synchronize()
            out = [r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy()]
            out += [x.cpu().numpy() for x in gcb] + [x.cpu().numpy() for x in r.grad_means]
            if ref is None:
                ref = out
                continue
            for a, b in zip(ref, out):
                np.testing.assert_array_equal(a, b)


def test_fused_scene_split_gradient_layout():
    """One shared codebook whose gradient is asked for as two blocks (the SR
    columns and the SH columns in separate arrays): the backward takes the
    two-codebook path (chain rule in Gaussian order, one row sort and
    reduction per block) after a forward that already ordered the Gaussians
    by row for the fused path.  Mean gradients are the same arithmetic in
    both kernels, so bitwise equal; the blocks equal the fused codebook
    gradient up to the order of the row sums; a fused-layout backward after
    it still reads the forward's row order and repeats the first one bit for
    bit."""
    wl = small_workload("clusters20k_d3")
    say("[split gradient layout] clusters20k_d3")
    r = gpu_renderer(wl)
    g = torch.from_numpy(np.random.default_rng(8).standard_normal((r.n_pixels, 3)).astype(np.float32) * 1e-5).cuda()
    r.forward()
    gm, gcb = r.backward(g)
    torch.cuda.synchronize()
    gm0, gcb0 = gm[0].cpu().numpy().copy(), gcb[0].cpu().numpy().copy()
    s = r.scenes[0]
    gsr = torch.full((s.k, 8), float("nan"), dtype=torch.float32, device="cuda")
    gsh = torch.full((s.k, s.r - 8), float("nan"), dtype=torch.float32, device="cuda")
    d = r._grads[0]
    saved = (d.sr, d.sr_stride, d.sr_col0, d.sh, d.sh_stride, d.sh_col0)
    d.sr, d.sr_stride, d.sr_col0 = gsr.data_ptr(), 8, 0
    d.sh, d.sh_stride, d.sh_col0 = gsh.data_ptr(), s.r - 8, 0
    try:
        gm, _ = r.backward(g)
        torch.cuda.synchronize()
        gm1 = gm[0].cpu().numpy().copy()
    finally:
        d.sr, d.sr_stride, d.sr_col0, d.sh, d.sh_stride, d.sh_col0 = saved
    np.testing.assert_array_equal(gm1, gm0)
    split = np.concatenate([gsr.cpu().numpy(), gsh.cpu().numpy()], 1)
    assert np.isfinite(split).all()
    e = rel_l2(split, gcb0)
    say(f"  split vs fused codebook gradient rel L2 {e:.2e}")
    assert e <= 1e-5
    gm, gcb = r.backward(g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(gm[0].cpu().numpy(), gm0)
    np.testing.assert_array_equal(gcb[0].cpu().numpy(), gcb0)


def _bin_inputs(seed, n, tx, ty, V, ties=True):
    rng = np.random.default_rng(seed)
    if ties:
        key = rng.integers(0x3E000000, 0x3E000100, n).astype(np.uint32)
    else:
        key = rng.integers(0x3E000000, 0x42000000, n).astype(np.uint32)
    x0 = rng.integers(0, tx, n); y0 = rng.integers(0, ty, n)
    x1 = np.minimum(tx, x0 + rng.integers(0, 4, n)); y1 = np.minimum(ty, y0 + rng.integers(0, 4, n))
    trect = np.stack([x0, y0, x1, y1], 1).astype(np.uint16)
    view = rng.integers(0, V, n).astype(np.int32)
    return key, trect, view


def _gpu_bin(key, trect, view, tx, ty, V, cap):
    n = key.shape[0]
    dk = torch.from_numpy(key.view(np.int32)).cuda()
    dt = torch.from_numpy(trect.view(np.int16)).cuda()
    dv = torch.from_numpy(view).cuda() if view is not None else None
    sk = torch.zeros(max(cap, 1), dtype=torch.int64, device="cuda")
    sg = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
    rg = torch.zeros(V * tx * ty * 2, dtype=torch.int32, device="cuda")
    info = torch.zeros(4, dtype=torch.int64, device="cuda")
    nb = cgs.bin_tiles_workspace_bytes(n, tx, ty, V, cap)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    cgs.bin_tiles(dk.data_ptr() if n else None, dt.data_ptr() if n else None, cgs.ptr(dv), n, tx, ty, V,
                  sk.data_ptr(), sg.data_ptr(), rg.data_ptr(), cap, info.data_ptr(), ws.data_ptr(), nb,
                  torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert cgs.load().cgs_sort_stalls() == 0
    return (sk.cpu().numpy().view(np.uint64), sg.cpu().numpy().view(np.uint32),
            rg.cpu().numpy().view(np.uint32).reshape(-1, 2), info.cpu().numpy())


@pytest.mark.parametrize("seed,n,tx,ty,V,ties", [(1, 5000, 13, 9, 3, True), (2, 20000, 40, 30, 1, False),
                                                 (3, 1, 4, 4, 1, True), (4, 0, 4, 4, 2, True),
                                                 (5, 70000, 123, 69, 4, True), (6, 300000, 123, 69, 4, False)])
def test_bin_tiles_bit_exact(seed, n, tx, ty, V, ties):
    say(f"[bin_tiles] seed={seed} n={n} tiles={tx}x{ty}x{V}")
    key, trect, view = _bin_inputs(seed, n, tx, ty, V, ties)
    osk, osg, orng = oracle.bin_tiles(key, trect, view, tx, ty, V)
    M = osk.shape[0]
    sk, sg, rg, info = _gpu_bin(key, trect, view, tx, ty, V, M + 7)
    assert info[0] == 0 and info[1] == M
    np.testing.assert_array_equal(sk[:M], osk)
    np.testing.assert_array_equal(sg[:M], osg)
    np.testing.assert_array_equal(rg, orng)


def test_bin_tiles_capacity_overflow():
    say("[bin_tiles] capacity overflow")
    key, trect, view = _bin_inputs(9, 3000, 10, 10, 2)
    osk, _, _ = oracle.bin_tiles(key, trect, view, 10, 10, 2)
    M = osk.shape[0]
    _, _, rg, info = _gpu_bin(key, trect, view, 10, 10, 2, M - 1)
    assert info[0] == cgs.CGS_ECAPACITY and info[1] == M
    assert (rg[:, 0] == rg[:, 1]).all()


def _gpu_reduce(g, idx, k, perm=None, ld_out=None):
    n, d = g.shape
    ld_out = ld_out or d
    dg = torch.from_numpy(np.ascontiguousarray(g, np.float32)).cuda()
    di = torch.from_numpy(np.ascontiguousarray(idx, np.int32)).cuda()
    dp = torch.from_numpy(np.ascontiguousarray(perm, np.int32)).cuda() if perm is not None else None
    out = torch.full((k, ld_out), 7.0, dtype=torch.float32, device="cuda")
    nb = cgs.codebook_grad_reduce_workspace_bytes(n, k, d)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    cgs.codebook_grad_reduce(dg.data_ptr() if n else None, d, di.data_ptr() if n else None, cgs.ptr(dp), n, k, d,
                             out.data_ptr(), ld_out, ws.data_ptr(), nb, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("case", ["uniform", "zipf", "identity", "single_row", "empty_rows", "wide", "perm",
                                  "empty"])
def test_codebook_grad_reduce(case):
    say(f"[codebook_grad_reduce] {case}")
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    n, k, d = 50000, 4096, 56
    if case == "zipf":
        idx = np.minimum(rng.zipf(1.1, n) - 1, k - 1)
    elif case == "identity":
        n = k = 3000
        idx = np.arange(n)
    elif case == "single_row":
        k = 1
        idx = np.zeros(n, int)
    elif case == "empty_rows":
        idx = rng.integers(0, k // 4, n) * 4
    elif case == "wide":
        n, d = 9000, 130
        idx = rng.integers(0, 300, n)
        k = 300
    elif case == "empty":
        n = 0
        idx = np.zeros(0, int)
    else:
        idx = rng.integers(0, k, n)
    g = rng.standard_normal((n, d)).astype(np.float32)
    perm = np.argsort(idx, kind="stable") if case == "perm" else None
    got = _gpu_reduce(g, idx, k, perm)
    ref = oracle.codebook_grad_reduce(g.astype(np.float64), idx, k)
    scale = np.sqrt(np.bincount(idx, minlength=k) + 1.0)[:, None]
    assert np.abs(got - ref).max() <= 1e-5 * scale.max() * 4, np.abs(got - ref).max()
    if case == "identity":
        np.testing.assert_array_equal(got, g)


def test_loss_l1():
    say("[loss_l1]")
    rng = np.random.default_rng(3)
    n = 3 * 1000 * 777 + 5
    a = rng.uniform(0, 1, n).astype(np.float32)
    b = rng.uniform(0, 1, n).astype(np.float32)
    b[:100] = a[:100]
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    grad = torch.empty_like(da)
    loss = torch.zeros(1, device="cuda")
    ws = torch.empty(cgs.loss_l1_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    render.loss_l1(da, db, grad, loss, ws)
    torch.cuda.synchronize()
    L, g = oracle.loss_l1(a, b)
    assert abs(loss.item() - L) <= 1e-6 * L
    np.testing.assert_array_equal(grad.cpu().numpy(), g.astype(np.float32))


@pytest.mark.parametrize("bf16", [False, True])
def test_two_codebook_layout(bf16):
    """The paper's state (Sec. 4.1): SR codebook [|SR|, 7], SH codebook
    [|SH|, 48], indices g2sr / g2sh, per-Gaussian opacity; two segmented
    reductions plus a per-Gaussian opacity gradient."""
    say(f"[two codebooks] bf16={bf16}")
    rng = np.random.default_rng(91 + int(bf16))
    n, ksr, ksh, d = 15000, 300, 700, 3
    W, H = 160, 120
    means = sc.clustered_means(rng, n).astype(np.float32)
    sr = np.zeros((ksr, 7))
    sr[:, 0:3] = rng.normal(sc.screen_matched_mu(W), 0.5, (ksr, 3))
    q = rng.standard_normal((ksr, 4))
    sr[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    sh = np.zeros((ksh, 48))
    sh[:, 0:3] = rng.uniform(0, 1, (ksh, 3))
    sh[:, 3:] = rng.normal(0, 0.05, (ksh, 45))
    sr32, sh32 = sr.astype(np.float32), sh.astype(np.float32)
    if bf16:
        sr_bits, sh_bits = sc.f32_to_bf16_bits(sr32), sc.f32_to_bf16_bits(sh32)
        sr32, sh32 = sc.bf16_bits_to_f32(sr_bits), sc.bf16_bits_to_f32(sh_bits)
    logit = rng.standard_normal(n).astype(np.float32)
    g2sr = rng.integers(0, ksr, n).astype(np.int32)
    g2sh = rng.integers(0, ksh, n).astype(np.int32)
    cam = sc.pinhole(W, H, (0.3, -0.2, -3.0))
    target = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    rows = np.concatenate([sr32[g2sr], logit[:, None], sh32[g2sh]], 1).astype(np.float32)
    host = sc.Scene(means, np.zeros(n, np.int32), np.zeros((1, 56), np.float32), d)
    pix = full_pixels(cam)
    base = oracle.render_view(host, cam, pix, rows32=rows)
    L, g = oracle.loss_l1(base["color"].reshape(H, W, 3), target)
    g = g.reshape(-1, 3)
    g[base["ambiguous"]] = 0.0
    g32 = g.astype(np.float32)
    og = oracle.render_view(host, cam, pix, grad_color=g32.astype(np.float64), rows32=rows)
    o_sr = oracle.codebook_grad_reduce(og["grad_rows"][:, :7], g2sr, ksr)
    o_sh = oracle.codebook_grad_reduce(og["grad_rows"][:, 8:], g2sh, ksh)
    o_op = og["grad_rows"][:, 7]

    def dev(a, dt=None):
        t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
        return t
    if bf16:
        dsr = dev(sr_bits.view(np.int16)).view(torch.bfloat16)
        dsh = dev(sh_bits.view(np.int16)).view(torch.bfloat16)
    else:
        dsr, dsh = dev(sr32), dev(sh32)
    ds = render.DeviceScene2(dev(means), dev(g2sr), dev(g2sh), dsr, dsh, dev(logit), d)
    r = render.Renderer([ds], [cam], [0])
    r.fit_capacity()
    r.forward()
    torch.cuda.synchronize()
    ec, et, mism, namb = compare_view(r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy(), cam,
                                      pix, base)
    say(f"  colour err {ec:.2e} T err {et:.2e} n_last mismatches {mism} ambiguous {namb}")
    assert ec <= IMAGE_TOL and et <= IMAGE_TOL and mism == 0
    r.backward(torch.from_numpy(g32).cuda())
    torch.cuda.synchronize()
    errs = {"means": rel_l2(r.grad_means[0].cpu().numpy(), og["grad_means"]),
            "sr": rel_l2(r.grad_sr[0].cpu().numpy(), o_sr),
            "sh": rel_l2(r.grad_sh[0].cpu().numpy(), o_sh),
            "opacity": rel_l2(r.grad_opacity[0].cpu().numpy(), o_op)}
    say("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def test_needle_gaussians_fp64_island():
    """Needle Gaussians (long axis 2000x the short ones, 30-60 degrees on
    screen, 35-90 px long sigma) whose projected 2x2 covariance is so
    elongated that a c - b^2 cancels: the conic then comes from the FP64
    determinant and inverse.  The host checks with the oracle's FP64 Sigma2D
    that every needle has det <= 0.7 * 2^-10 a c (inside the island with room
    for FP32 rounding of a, b, c), then compares the image and gradients.

    Error model (the known limit of the island: it removes the cancellation
    in the determinant, not the rounding already in the FP32 a, b, c).  a, b, c
    come out of an FP32 chain of about 40 roundings (quaternion, rotation,
    R S, Sigma, J W Sigma W^T J^T); by the probabilistic rounding-error bound
    (Higham and Mary, SIAM J. Sci. Comput. 41, 2019) their error is about
    sqrt(40) u relative to lambda_max, taken as EPS = 8u = 2^-21 (u = 2^-24).
    The determinant, the FP32 conic entries and the FP32 quadratic form along
    the needle each turn that into a relative error of the power of about
    kappa EPS (2 + 3 + 1 terms; kappa = lambda_max / lambda_min of Sigma2D):
    |d power| <= 6 kappa EPS |power|.  Hence, per needle:
      - alpha's decision against 1/255 (|power| <= ln(255 * 0.99)) is
        ambiguous within a relative margin of 6 ln(252.45) kappa EPS, passed
        to the oracle as that Gaussian's margin (it also widens every
        transmittance test after it);
      - alpha's error is <= 6 kappa EPS max_p(o e^p |p|) <= 2.21 kappa EPS, and
        colour and T move by at most that (|c - behind| <= 1 here): pixels of
        tiles in needle rectangles are held to 1e-4 + sum over those needles
        of 3 kappa EPS, every other pixel to 1e-4;
      - a needle's gradient (a sum of per-pixel terms each off by at most
        6 kappa EPS |power| <= 33 kappa EPS, plus 2 kappa EPS through the
        derivative of the inverse) to 36 kappa EPS relative L2; the
        background Gaussians' blocks to 1e-3.
    The measured errors are printed and recorded."""
    say("[needles] FP64 determinant island")
    EPS = 2.0 ** -21
    s = sc.needle_scene(5)
    cam = sc.pinhole(320, 240, (0.0, 0.0, -3.0))
    rng = np.random.default_rng(31)
    wl = sc.Workload("needles", [s], [cam], np.array([0], np.int32),
                     [rng.uniform(0, 1, (240, 320, 3)).astype(np.float32)], False)
    n_needle = 12
    nd = np.arange(s.n - n_needle, s.n)
    rows = oracle.decode_rows(s).astype(np.float64)
    pr = oracle.project(torch.tensor(s.means[nd].astype(np.float64)), torch.tensor(rows[nd]), cam, s.sh_degree)
    S2 = pr["Sigma2D"].numpy()
    a, b, c = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
    ratio = (a * c - b * b) / (a * c)
    lam = np.linalg.eigvalsh(S2)
    kappa = lam[:, 1] / lam[:, 0]
    say("  det/(ac): " + " ".join(f"{x:.1e}" for x in ratio))
    say("  kappa: " + " ".join(f"{x:.0f}" for x in kappa))
    assert (ratio <= 0.7 * 2.0 ** -10).all()
    # per-pixel bound from the needles whose tile rectangle holds the pixel
    _, trect, kept = oracle.keyspec(s.means[nd], rows[nd, :7].astype(np.float32), cam)
    assert kept.all()
    W, H = cam.width, cam.height
    ksum = np.zeros((H, W))
    for i in range(n_needle):
        x0, y0, x1, y1 = (int(t) for t in trect[i])
        ksum[16 * y0:16 * y1, 16 * x0:16 * x1] += kappa[i]
    tol = IMAGE_TOL + 3.0 * EPS * ksum
    rec_margin = np.zeros(s.n)
    rec_margin[nd] = 6.0 * np.log(255.0 * 0.99) * kappa * EPS
    r = gpu_renderer(wl)
    r.forward()
    torch.cuda.synchronize()
    pix = full_pixels(cam)
    base = oracle.render_view(s, cam, pix, rec_margin=rec_margin)
    img = r.image.cpu().numpy().astype(np.float64)
    err = np.abs(img - base["color"]).max(1)
    terr = np.abs(r.T_final.cpu().numpy().astype(np.float64) - base["T"])
    ok = ~base["ambiguous"]
    t_flat = tol.ravel()
    in_needle = ksum.ravel() > 0
    nl = r.n_last.cpu().numpy()
    mism = int((nl[ok] != base["n_last"][ok]).sum())
    worst_img = float((err[ok] / t_flat[ok]).max())
    say(f"  image: max err off needles {err[ok & ~in_needle].max():.2e}, on needles {err[ok & in_needle].max():.2e} "
        f"(bound there {t_flat[ok & in_needle].min():.2e}..{t_flat[ok & in_needle].max():.2e}), "
        f"max err / bound {worst_img:.3f}, T max err / bound {(terr[ok] / t_flat[ok]).max():.3f}, "
        f"n_last mismatches {mism}, ambiguous {(~ok).sum()} of {len(pix)}")
    assert (err[ok] <= t_flat[ok]).all()
    assert (terr[ok] <= t_flat[ok]).all()
    assert mism == 0
    assert (~ok).sum() <= 0.02 * len(pix)
    # gradients
    gcols, gfull = oracle_grad_image(wl, [pix], [base])
    outs = [oracle.render_view(s, cam, pix, grad_color=gcols[0], rec_margin=rec_margin)]
    ogm, ogcb = oracle_scene_grads(wl, outs)
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    gm, gcb = gm[0].cpu().numpy(), gcb[0].cpu().numpy()
    kb = s.k - n_needle
    bg_err = grad_errors(gm[:s.n - n_needle], gcb[:kb], ogm[0][:s.n - n_needle], ogcb[0][:kb])
    say("  background: " + " ".join(f"{k}={v:.2e}" for k, v in bg_err.items()))
    for k, e in bg_err.items():
        assert e <= GRAD_TOL, (k, e)
    worst = 0.0
    needle_errs = []
    for i in range(n_needle):
        er = rel_l2(gcb[kb + i], ogcb[0][kb + i])
        em = rel_l2(gm[nd[i]], ogm[0][nd[i]])
        bound = 36.0 * EPS * kappa[i]
        worst = max(worst, max(er, em) / bound)
        needle_errs.append((float(kappa[i]), er, em))
        blk = " ".join(f"{k}={rel_l2(gcb[kb + i][sl], ogcb[0][kb + i][sl]):.1e}"
                       for k, sl in BLOCKS.items() if ogcb[0][kb + i][sl].size)
        say(f"  needle {i}: kappa {kappa[i]:.0f} row rel err {er:.2e} mean rel err {em:.2e} (bound {bound:.2e}) [{blk}]")
        assert er <= bound and em <= bound, (i, er, em, bound)
    record("needles_fp64_island", kappa_min=float(kappa.min()), kappa_max=float(kappa.max()),
           det_ratio_max=float(ratio.max()), image_err_needle=float(err[ok & in_needle].max()),
           image_err_other=float(err[ok & ~in_needle].max()), image_err_over_bound=worst_img,
           ambiguous=int((~ok).sum()), pixels=len(pix),
           row_rel_l2_max=max(e[1] for e in needle_errs), mean_rel_l2_max=max(e[2] for e in needle_errs),
           grad_err_over_bound=worst, background=bg_err)
    say(f"  needle gradients: worst error / bound {worst:.2f}")


def test_out_of_range_indices_are_absent():
    """A Gaussian whose codebook index lies outside its codebook (negative or
    >= K) is invalid: nothing renders it and its gradients are zero.  A
    two-scene batch holding 40 such Gaussians per scene must render and
    differentiate as the oracle's batch without them; the single-codebook
    backward, which walks Gaussians sorted by row, keeps each of them in its
    own scene's rows (the other scene's rows are untouched)."""
    rng = np.random.default_rng(91)
    ss = [sc.make_scene(rng, n, k, 3, sc.screen_matched_mu(64), clusters=True) for n, k in ((3000, 64), (2000, 100))]
    bad, keep = [], []
    for s in ss:
        b = np.sort(rng.choice(s.n, 40, replace=False))
        s.idx[b[:20]] = (-1 - rng.integers(0, 5, 20)).astype(np.int32)
        s.idx[b[20:]] = (s.k + rng.integers(0, 5, 20)).astype(np.int32)
        bad.append(b)
        keep.append(np.setdiff1d(np.arange(s.n), b))
    cams = [sc.pinhole(64, 48, (0.0, 0.0, -3.0)), sc.pinhole(64, 64, (0.3, 0.0, -3.0))]
    tg = [rng.uniform(0, 1, (c.height, c.width, 3)).astype(np.float32) for c in cams]
    vs = np.array([0, 1], np.int32)
    wl = sc.Workload("oob_idx", ss, cams, vs, tg, False)
    ref = sc.Workload("oob_idx_ref", [sc.Scene(s.means[k], s.idx[k], s.cb, s.sh_degree) for s, k in zip(ss, keep)],
                      cams, vs, tg, False)
    say("[out-of-range indices] 2 scenes, 40 invalid Gaussians each")
    r = gpu_renderer(wl)
    r.forward()
    torch.cuda.synchronize()
    img, T, nl = r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy()
    pix = [full_pixels(c) for c in cams]
    base = oracle_render(ref, pix)
    for v, cam in enumerate(cams):
        a, b = r.pix_off[v], r.pix_off[v + 1]
        ec, et, mism, namb = compare_view(img[a:b], T[a:b], nl[a:b], cam, pix[v], base[v])
        say(f"  view {v}: colour err {ec:.2e} T err {et:.2e} n_last mismatches {mism} ambiguous {namb}")
        assert ec <= IMAGE_TOL and et <= IMAGE_TOL and mism == 0
    gcols, gfull = oracle_grad_image(ref, pix, base)
    ogm, ogcb = oracle_scene_grads(ref, oracle_render(ref, pix, gcols))
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    for i in range(len(ss)):
        m = gm[i].cpu().numpy()
        assert np.all(m[bad[i]] == 0.0)
        errs = grad_errors(m[keep[i]], gcb[i].cpu().numpy(), ogm[i], ogcb[i])
        say(f"  scene {i}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        for k, e in errs.items():
            assert e <= GRAD_TOL, (k, e)


def _depth_range_workload(kind: str) -> sc.Workload:
    """Scenes whose live depth keys span 0 bits (every mean on the plane
    z = 0, camera axis-aligned at z = -3: all camera depths exactly 3.0, so
    every key ties), about 2^18 (depths 3 to 3.05) and more than 2^27 (depths
    0.3 to 1e5): the depth sort takes 1, 2 and 4 passes of 9 bits."""
    rng = np.random.default_rng({"flat": 81, "shallow": 82, "deep": 83}[kind])
    s = sc.make_scene(rng, 4000, 128, 3, sc.screen_matched_mu(96), clusters=False)
    means = s.means.copy()
    if kind == "flat":
        means[:, 2] = 0.0
    elif kind == "shallow":
        means[:, 2] = rng.uniform(0.0, 0.05, means.shape[0]).astype(np.float32)
    else:
        dist = np.exp(rng.uniform(np.log(0.3), np.log(1e5), means.shape[0]))
        means[:, 2] = (dist - 3.0).astype(np.float32)
        means[:, 0:2] *= (dist / 3.0)[:, None].astype(np.float32)      # keep them in the frustum
    s = sc.Scene(means, s.idx, s.cb, 3)
    cams = [sc.pinhole(96, 72, (0.0, 0.0, -3.0))]
    return sc.Workload("depth_" + kind, [s], cams, np.array([0], np.int32),
                       [rng.uniform(0, 1, (72, 96, 3)).astype(np.float32)], False)


@pytest.mark.parametrize("kind", ["flat", "shallow", "deep"])
def test_depth_range_pass_counts(kind):
    wl = _depth_range_workload(kind)
    say(f"[depth range] {kind}")
    r = gpu_renderer(wl)
    r.forward()
    torch.cuda.synchronize()
    img, T, nl = r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy()
    pix = [full_pixels(c) for c in wl.cameras]
    base = oracle_render(wl, pix)
    ec, et, mism, namb = compare_view(img, T, nl, wl.cameras[0], pix[0], base[0])
    say(f"  colour err {ec:.2e} T err {et:.2e} n_last mismatches {mism} ambiguous {namb}")
    assert ec <= IMAGE_TOL and et <= IMAGE_TOL and mism == 0
    assert namb <= 0.01 * len(pix[0])
    gcols, gfull = oracle_grad_image(wl, pix, base)
    ogm, ogcb = oracle_scene_grads(wl, oracle_render(wl, pix, gcols))
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    errs = grad_errors(gm[0].cpu().numpy(), gcb[0].cpu().numpy(), ogm[0], ogcb[0])
    say("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def test_more_than_65536_tiles():
    """A batch of five 2400 x 1600 views (75 000 tiles, fewer than 256 per
    side): instance tile keys need 17 bits, so binning keeps 32-bit keys
    (batches of at most 65536 tiles store them in 16 bits).  Forward and
    backward against the oracle on 24 random tiles per view."""
    rng = np.random.default_rng(95)
    s = sc.make_scene(rng, 6000, 256, 1, sc.screen_matched_mu(2400), clusters=True)
    cams = [sc.pinhole(2400, 1600, (3.0 * np.sin(a), 0.3, -3.0 * np.cos(a))) for a in (0.0, 1.2, 2.4, 3.6, 4.8)]
    tg = [rng.uniform(0, 1, (c.height, c.width, 3)).astype(np.float32) for c in cams]
    wl = sc.Workload("tiles75k", [s], cams, np.zeros(5, np.int32), tg, False)
    say("[more than 65536 tiles] 5 x 2400 x 1600")
    r = gpu_renderer(wl)
    r.forward()
    torch.cuda.synchronize()
    img, T, nl = r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy()
    pix = [random_tiles(c, 24, 950 + v) for v, c in enumerate(cams)]
    base = oracle_render(wl, pix)
    for v, cam in enumerate(cams):
        a, b = r.pix_off[v], r.pix_off[v + 1]
        ec, et, mism, namb = compare_view(img[a:b], T[a:b], nl[a:b], cam, pix[v], base[v])
        say(f"  view {v}: colour err {ec:.2e} T err {et:.2e} n_last mismatches {mism} ambiguous {namb}")
        assert ec <= IMAGE_TOL and et <= IMAGE_TOL and mism == 0
    gcols, gfull = oracle_grad_image(wl, pix, base)
    ogm, ogcb = oracle_scene_grads(wl, oracle_render(wl, pix, gcols))
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    errs = grad_errors(gm[0].cpu().numpy(), gcb[0].cpu().numpy(), ogm[0], ogcb[0])
    say("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


@pytest.mark.parametrize("k", [1, 2])
def test_tiny_codebook_rows_span_many_wavefronts(k):
    """20 000 Gaussians sharing 1 or 2 codebook rows: in the fused chain rule
    and reduction each row spans hundreds of wavefronts of the row-sorted
    order, so its gradient is the merge of as many partial rows."""
    rng = np.random.default_rng(97 + k)
    s = sc.make_scene(rng, 20000, k, 3, sc.screen_matched_mu(160), clusters=True)
    cams = [sc.pinhole(160, 120, (0.2, -0.1, -3.0))]
    wl = sc.Workload(f"k{k}", [s], cams, np.array([0], np.int32),
                     [rng.uniform(0, 1, (120, 160, 3)).astype(np.float32)], False)
    say(f"[tiny codebook] K = {k}, N = 20000")
    r = gpu_renderer(wl)
    pix = [full_pixels(c) for c in cams]
    base = oracle_render(wl, pix)
    gcols, gfull = oracle_grad_image(wl, pix, base)
    ogm, ogcb = oracle_scene_grads(wl, oracle_render(wl, pix, gcols))
    r.forward()
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    errs = grad_errors(gm[0].cpu().numpy(), gcb[0].cpu().numpy(), ogm[0], ogcb[0])
    say("  " + " ".join(f"{kk}={v:.2e}" for kk, v in errs.items()))
    for kk, e in errs.items():
        assert e <= GRAD_TOL, (kk, e)
