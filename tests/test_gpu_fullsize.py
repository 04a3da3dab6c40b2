"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (all views of a workload in one batched call).

The GPU renders every pixel; the oracle renders a random sample of 16x16
tiles (what it can afford one by one) and the gradient check uses a loss
restricted to those tiles on both sides.  Properties that hold at any size
are checked on everything: the FP32 skeleton (depth keys, tile rectangles) of
every Gaussian in every view, and the binning (each tile lists exactly the
Gaussians whose rectangle holds it, in (depth, index) order)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2509_03775_amd import cgs, render, scenes as sc
from harness import (GRAD_TOL, IMAGE_TOL, compare_view, grad_error_stats, grad_errors, oracle_grad_image,
                     oracle_render, oracle_scene_grads, random_tiles, record, say)

pytestmark = pytest.mark.gpu

FULL = ["clusters200k_800px", "clusters1m_1600x1064", "clusters4m_bf16_4x1957x1091", "uneven16_512px"]
TILES_PER_VIEW = {"clusters200k_800px": 64, "clusters1m_1600x1064": 128, "clusters4m_bf16_4x1957x1091": 64,
                  "uneven16_512px": 8}

_cache = {}


def workload_and_renderer(name):
    if name not in _cache:
        _cache.clear()
        torch.cuda.empty_cache()
        say(f"  building {name}")
        wl = sc.make_workload(name)
        ds = [render.DeviceScene.from_host(s, bf16=wl.bf16) for s in wl.scenes]
        r = render.Renderer(ds, wl.cameras, wl.view_scene)
        m = r.fit_capacity()
        say(f"  {name}: {m} instances")
        _cache[name] = (wl, r)
    return _cache[name]


@pytest.mark.parametrize("name", FULL)
def test_skeleton_every_gaussian_bit_exact(name):
    say(f"[full skeleton] {name}")
    wl, r = workload_and_renderer(name)
    r.forward()
    torch.cuda.synchronize()
    lay = r.layout()
    R = lay.n_records
    ws = r.ws
    key = ws[lay.depth_key:lay.depth_key + 4 * R].view(torch.int32).cpu().numpy().view(np.uint32)
    tr = ws[lay.records:lay.records + 48 * R].view(torch.int32).view(R, 12)[:, 9:11].contiguous().cpu().numpy().view(np.uint32)
    off = 0
    for v, cam in enumerate(wl.cameras):
        s = wl.scenes[int(wl.view_scene[v])]
        rows = oracle.decode_rows(s)
        okey, otr, okept = oracle.keyspec(s.means, rows[:, :7], cam)
        gk, gt = key[off:off + s.n], tr[off:off + s.n]
        np.testing.assert_array_equal(gk != 0x7F800000, okept)
        np.testing.assert_array_equal(gk[okept], okey[okept])
        g4 = np.stack([gt[:, 0] & 0xFFFF, gt[:, 0] >> 16, gt[:, 1] & 0xFFFF, gt[:, 1] >> 16], 1)
        np.testing.assert_array_equal(g4[okept], otr[okept].astype(np.uint32))
        off += s.n


@pytest.mark.parametrize("name", FULL)
def test_binning_properties(name):
    """Every tile's list holds exactly the records whose rectangle contains
    the tile, sorted by (depth key, record index)."""
    say(f"[full binning] {name}")
    wl, r = workload_and_renderer(name)
    r.forward()
    torch.cuda.synchronize()
    lay = r.layout()
    R, T = lay.n_records, lay.n_tiles
    ws = r.ws
    M = r.instances()
    key = ws[lay.depth_key:lay.depth_key + 4 * R].view(torch.int32).cpu().numpy().view(np.uint32)
    tr = ws[lay.records:lay.records + 48 * R].view(torch.int32).view(R, 12)[:, 9:11].contiguous().cpu().numpy().view(np.uint32)
    rec = ws[lay.inst_rec:lay.inst_rec + 4 * M].view(torch.int32).cpu().numpy().view(np.uint32)
    rng_ = ws[lay.tile_range:lay.tile_range + 8 * T].view(torch.int32).cpu().numpy().view(np.uint32).reshape(T, 2)
    x0, y0 = (tr[:, 0] & 0xFFFF).astype(np.int64), (tr[:, 0] >> 16).astype(np.int64)
    x1, y1 = (tr[:, 1] & 0xFFFF).astype(np.int64), (tr[:, 1] >> 16).astype(np.int64)
    cnt = np.maximum(x1 - x0, 0) * np.maximum(y1 - y0, 0)
    assert int(cnt.sum()) == M
    assert rng_[0, 0] == 0 and rng_[-1, 1] == M and (rng_[1:, 0] == rng_[:-1, 1]).all()
    tile_of = np.repeat(np.arange(T), (rng_[:, 1] - rng_[:, 0]).astype(np.int64))
    # record's view -> tile coordinates inside the record's rectangle
    roff = np.array([0] + [int(wl.scenes[int(s)].n) for s in wl.view_scene]).cumsum()
    toff = np.array([0] + [((c.width + 15) // 16) * ((c.height + 15) // 16) for c in wl.cameras]).cumsum()
    txs = np.array([(c.width + 15) // 16 for c in wl.cameras])
    v = np.searchsorted(roff, rec, side="right") - 1
    lt = tile_of - toff[v]
    tx, ty = lt % txs[v], lt // txs[v]
    assert ((x0[rec] <= tx) & (tx < x1[rec]) & (y0[rec] <= ty) & (ty < y1[rec])).all()
    # order inside each tile: (depth key, record) strictly increasing
    same = tile_of[1:] == tile_of[:-1]
    k0, k1 = key[rec[:-1]].astype(np.int64), key[rec[1:]].astype(np.int64)
    inc = (k0 < k1) | ((k0 == k1) & (rec[:-1] < rec[1:]))
    assert inc[same].all()
    # no record listed twice in a tile; counts per record match its rectangle
    assert (np.bincount(rec, minlength=R) == cnt).all()


@pytest.mark.parametrize("name", FULL)
def test_sampled_image_and_gradients(name):
    say(f"[full sampled parity] {name}")
    wl, r = workload_and_renderer(name)
    r.forward()
    torch.cuda.synchronize()
    img, T, nl = r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy()
    pix = [random_tiles(c, TILES_PER_VIEW[name], 100 + v) for v, c in enumerate(wl.cameras)]
    base = oracle_render(wl, pix)
    views = []
    for v, cam in enumerate(wl.cameras):
        a, b = r.pix_off[v], r.pix_off[v + 1]
        ec, et, mism, namb = compare_view(img[a:b], T[a:b], nl[a:b], cam, pix[v], base[v])
        say(f"  view {v}: colour err {ec:.2e} T err {et:.2e} n_last mismatches {mism} ambiguous {namb}/{len(pix[v])}")
        views.append({"image_max_abs": ec, "T_max_abs": et, "ambiguous": namb, "pixels": int(len(pix[v]))})
        assert ec <= IMAGE_TOL and et <= IMAGE_TOL and mism == 0
        assert namb <= 0.02 * len(pix[v])
    gcols, gfull = oracle_grad_image(wl, pix, base)
    outs = oracle_render(wl, pix, gcols)
    ogm, ogcb = oracle_scene_grads(wl, outs)
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    scenes_rec = []
    for i in range(len(wl.scenes)):
        errs = grad_errors(gm[i].cpu().numpy(), gcb[i].cpu().numpy(), ogm[i], ogcb[i])
        scenes_rec.append(grad_error_stats(gm[i].cpu().numpy(), gcb[i].cpu().numpy(), ogm[i], ogcb[i]))
        say(f"  scene {i}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        for k, e in errs.items():
            assert e <= GRAD_TOL, (k, e)
    record(name, tiles_per_view=TILES_PER_VIEW[name], views=views, grads=scenes_rec)


def test_batched_equals_per_view_calls():
    """The uneven 16-scene batch in one call gives bitwise the per-scene
    results of separate calls (same kernels; every sum has a fixed order that
    does not depend on where a scene sits in the batch)."""
    name = "uneven16_512px"
    say(f"[batched vs plain] {name}")
    wl, r = workload_and_renderer(name)
    rng = np.random.default_rng(3)
    g = torch.from_numpy((rng.standard_normal((wl.n_pixels, 3)) * 1e-6).astype(np.float32)).cuda()
    r.forward()
    gm, gcb = r.backward(g)
    torch.cuda.synchronize()
    img = r.image.cpu().numpy()
    for v in range(0, len(wl.cameras), 5):
        s = int(wl.view_scene[v])
        r1 = render.Renderer([r.scenes[s]], [wl.cameras[v]], [0])
        r1.fit_capacity()
        a, b = r.pix_off[v], r.pix_off[v + 1]
        np.testing.assert_array_equal(r1.image.cpu().numpy(), img[a:b])
        gm1, gcb1 = r1.backward(g[a:b].contiguous())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(gcb1[0].cpu().numpy(), gcb[s].cpu().numpy())
        np.testing.assert_array_equal(gm1[0].cpu().numpy(), gm[s].cpu().numpy())


def test_graph_replay_matches_eager():
    """forward + L1 + backward captured once in a HIP graph; three replays
    (with eager work in between) equal the eager step bit for bit.  The whole
    workspace is overwritten with garbage before each replay, so every value
    a replay reads (including what the library's second stream computes) must
    come from the graph itself."""
    name = "uneven16_512px"
    say(f"[graph replay] {name}")
    wl, r = workload_and_renderer(name)
    tgt = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).cuda()
    grad = torch.empty_like(tgt)
    loss = torch.zeros(1, device="cuda")
    lws = torch.empty(cgs.loss_l1_workspace_bytes(tgt.numel()), dtype=torch.uint8, device="cuda")

    def step():
        img = r.forward()
        render.loss_l1(img, tgt, grad, loss, lws)
        r.backward(grad)

    step()
    torch.cuda.synchronize()
    ref = (r.image.cpu().numpy().copy(), loss.cpu().numpy().copy(), [c.cpu().numpy().copy() for c in r.grad_cb],
           [m.cpu().numpy().copy() for m in r.grad_means])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        r.image.zero_()
        for c in r.grad_cb:
            c.zero_()
        for m in r.grad_means:
            m.zero_()
        r.ws.fill_(0x5A)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(r.image.cpu().numpy(), ref[0])
        np.testing.assert_array_equal(loss.cpu().numpy(), ref[1])
        for a, b in zip(r.grad_cb, ref[2]):
            np.testing.assert_array_equal(a.cpu().numpy(), b)
        for a, b in zip(r.grad_means, ref[3]):
            np.testing.assert_array_equal(a.cpu().numpy(), b)
        step()          # eager work between replays
        torch.cuda.synchronize()


def test_autograd_and_finite_differences_1m():
    """The 1M-Gaussian workload through torch.autograd (transmittance
    recomputed in the backward): gradients equal the direct backward call and
    agree with central finite differences (h = 1e-3) of the FP64 oracle loss
    on 64 random codebook entries, and with the oracle's gradient."""
    name = "clusters1m_1600x1064"
    say(f"[autograd + FD] {name}")
    wl, r = workload_and_renderer(name)
    s = wl.scenes[0]
    cam = wl.cameras[0]
    pix = random_tiles(cam, 64, 7)
    base = oracle.render_view(s, cam, pix, want_lists=True)
    gcol = np.zeros_like(base["color"])
    tgt = wl.targets[0][pix[:, 1], pix[:, 0]].astype(np.float64)
    gcol[:] = np.sign(base["color"] - tgt) / (3.0 * wl.n_pixels)
    gcol[base["ambiguous"]] = 0.0
    gfull = np.zeros((wl.n_pixels, 3), np.float32)
    gfull[pix[:, 1].astype(np.int64) * cam.width + pix[:, 0]] = gcol.astype(np.float32)
    gcol = gcol.astype(np.float32).astype(np.float64)
    # autograd path
    dsc = r.scenes[0]
    dsc.means.requires_grad_(True)
    dsc.cb.requires_grad_(True)
    img = render.render(r)
    img.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    ag_cb = dsc.cb.grad.cpu().numpy().astype(np.float64)
    ag_m = dsc.means.grad.cpu().numpy().astype(np.float64)
    dsc.means.requires_grad_(False)
    dsc.cb.requires_grad_(False)
    dsc.means.grad = None
    dsc.cb.grad = None
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ag_cb, gcb[0].cpu().numpy())
    np.testing.assert_array_equal(ag_m, gm[0].cpu().numpy())
    # oracle gradient
    og = oracle.render_view(s, cam, pix, grad_color=gcol)
    ogcb = oracle.codebook_grad_reduce(og["grad_rows"], s.idx, s.k)
    errs = grad_errors(ag_m, ag_cb, og["grad_means"], ogcb)
    say("  vs oracle: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)
    # finite differences of the oracle loss sum(g . C) on 64 entries that
    # some Gaussian rendered into the sampled tiles references
    fz = base["frozen"]
    used = np.unique(s.idx[fz["order"][np.unique(fz["fz_rec"])]])
    rng = np.random.default_rng(11)
    entries = rng.choice(used, size=min(64, used.size), replace=False)
    rows = oracle.decode_rows(s).astype(np.float64)     # per-Gaussian rows, perturbed in place
    h = 1e-3
    worst = 0.0
    for k in entries:
        d = rng.standard_normal(s.r)
        d /= np.linalg.norm(d)
        sel = np.nonzero(s.idx == k)[0]
        base_row = rows[sel[0]].copy()

        def L(sign):
            rows[sel] = base_row + sign * h * d
            o = oracle.render_view(s, cam, pix, frozen=fz, rows32=rows)
            return float((o["color"] * gcol).sum())

        fd = (L(1) - L(-1)) / (2 * h)
        rows[sel] = base_row
        an = float(ag_cb[k] @ d)
        ora = float(ogcb[k] @ d)
        scale = max(abs(fd), 1e-3 * np.linalg.norm(ogcb[k]) + 1e-12)
        err = abs(an - fd) / scale
        worst = max(worst, err)
        assert abs(ora - fd) <= 1e-4 * scale + 1e-12, (k, ora, fd)
        assert err <= 2e-3, (k, an, fd)
    say(f"  {len(entries)}-entry FD: worst relative difference GPU vs FD {worst:.2e}")


def test_sort_waits_never_hit_bound():
    """The radix passes' look-back waits (bounded so a pass always ends)
    never reached their bound in any call of this session's full-size runs."""
    assert cgs.load().cgs_sort_stalls() == 0


def test_uncompressed_identity_rows_1m():
    """The uncompressed baseline (one codebook row per Gaussian: K = N = 1M,
    identity indices, the per-Gaussian parameter layout of the paper's MCMC
    comparison): the row sort takes three radix passes (20-bit keys) and every
    row's reduction is a single Gaussian.  Image and n_last on 64 random tiles,
    and the gradient of every row against the oracle's per-Gaussian gradient."""
    name = "clusters1m_1600x1064"
    say(f"[uncompressed K = N] {name}")
    _cache.clear()
    torch.cuda.empty_cache()
    wl = sc.make_workload(name)
    s = wl.scenes[0]
    su = sc.Scene(s.means, np.arange(s.n, dtype=np.int32), np.ascontiguousarray(s.cb[s.idx]), s.sh_degree)
    wlu = sc.Workload(name + ":uncompressed", [su], wl.cameras, wl.view_scene, wl.targets, False)
    r = render.Renderer([render.DeviceScene.from_host(su)], wlu.cameras, wlu.view_scene)
    r.fit_capacity()
    r.forward()
    torch.cuda.synchronize()
    cam = wlu.cameras[0]
    pix = [random_tiles(cam, 64, 41)]
    base = oracle_render(wlu, pix)
    ec, et, mism, namb = compare_view(r.image.cpu().numpy(), r.T_final.cpu().numpy(), r.n_last.cpu().numpy(), cam,
                                      pix[0], base[0])
    say(f"  colour err {ec:.2e} T err {et:.2e} n_last mismatches {mism} ambiguous {namb}/{len(pix[0])}")
    assert ec <= IMAGE_TOL and et <= IMAGE_TOL and mism == 0
    gcols, gfull = oracle_grad_image(wlu, pix, base)
    outs = oracle_render(wlu, pix, gcols)
    gm, gcb = r.backward(torch.from_numpy(gfull).cuda())
    torch.cuda.synchronize()
    gcb, gm = gcb[0].cpu().numpy(), gm[0].cpu().numpy()
    errs = grad_errors(gm, gcb, outs[0]["grad_means"], outs[0]["grad_rows"])
    say("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)
    # rows of Gaussians no sampled pixel depends on are exactly zero
    untouched = np.abs(outs[0]["grad_rows"]).max(1) == 0
    assert untouched.sum() > 0.5 * s.n
    assert (gcb[untouched] == 0).all()
    record(name + ":uncompressed", views=[{"image_max_abs": ec, "T_max_abs": et, "ambiguous": namb,
                                           "pixels": int(len(pix[0]))}],
           grads=[grad_error_stats(gm, gcb, outs[0]["grad_means"], outs[0]["grad_rows"])])
