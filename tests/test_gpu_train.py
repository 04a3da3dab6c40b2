"""Parity of the training-step pieces with the oracle, through the C-ABI:
the SGLD noise generator (Philox words bit for bit, normals within FP32
rounding), the reconstruction loss of Eq. 4 with its SSIM term, and the SGLD
parameter update fused into the backward (fused FP32 in place, fused BF16
with an FP32 master and refreshed BF16 copy, the paper's two-codebook layout
with per-Gaussian opacity)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import train as otrain
from paper_2509_03775_amd import cgs, render, scenes as sc
from harness import (GRAD_TOL, full_pixels, oracle_grad_image, oracle_render, oracle_scene_grads, rel_l2, say)
from test_gpu_parity import gpu_renderer, small_workload

pytestmark = pytest.mark.gpu

NORMAL_TOL = 2e-5     # |z_gpu - z_oracle|: FP32 log / sqrt / sincospi against FP64 (|z| < 5.8)
LOSS_TOL = 1e-5       # relative error of the loss (FP32 window sums, FP64 totals)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cgs.load()
    yield
    torch.cuda.synchronize()


def test_sgld_normals():
    n, index0, tag, step, seed = 5000, (1 << 32) - 1234, 0x10003, 77, 0x0123456789ABCDEF
    say(f"[normals] n={n} index0={index0}")
    z = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    w = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    cgs.sgld_normals(n, index0, tag, step, seed, z.data_ptr(), w.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    idx = np.arange(n, dtype=np.uint64) + np.uint64(index0)
    ctr = np.stack([(idx & np.uint64(0xFFFFFFFF)).astype(np.uint32), (idx >> np.uint64(32)).astype(np.uint32),
                    np.full(n, tag, np.uint32), np.full(n, step, np.uint32)], 1)
    ref_w = otrain.philox4x32(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    assert np.array_equal(w.cpu().numpy().view(np.uint32), ref_w)
    err = np.abs(z.cpu().numpy().astype(np.float64) - otrain.normals(idx, tag, step, seed)).max()
    say(f"  max normal error {err:.2e}")
    assert err <= NORMAL_TOL


def _anticorrelated(h, w):
    """Image and target that are mirror images about 0.5 with a checkerboard
    of amplitude sqrt(C2 / 2): the local covariance is about -C2 / 2, so the
    SSIM factor 2 sxy + C2 passes through zero."""
    a = np.sqrt(otrain.SSIM_C2 / 2.0)
    cb = np.indices((h, w)).sum(0) % 2 * 2.0 - 1.0
    x = np.repeat((0.5 + a * cb)[:, :, None], 3, 2)
    y = np.repeat((0.5 - a * cb)[:, :, None], 3, 2)
    x[:, :, 1] = 0.3 + 0.9 * a * cb     # other channels near, not at, the zero
    return x.astype(np.float32), y.astype(np.float32)


@pytest.mark.parametrize("case", ["random", "anticorrelated"])
@pytest.mark.parametrize("lam", [0.0, 0.2, 1.0])
def test_loss_recon(lam, case):
    rng = np.random.default_rng(31)
    hw = [(37, 53), (16, 16), (1, 1), (70, 33)]
    say(f"[loss] lambda={lam} {case} views={hw}")
    if case == "random":
        ims = [rng.uniform(0, 1, (h, w, 3)).astype(np.float32) for h, w in hw]
        tgs = [np.clip(im + 0.15 * rng.standard_normal(im.shape), 0, 1).astype(np.float32) for im in ims]
        tgs[0][3, 4] = ims[0][3, 4]          # exact ties: sign(0) = 0 on both sides
    else:
        pairs = [_anticorrelated(h, w) for h, w in hw]
        ims, tgs = [p[0] for p in pairs], [p[1] for p in pairs]
    loss_o, grads_o = otrain.loss_recon(ims, tgs, lam)
    img = torch.from_numpy(np.concatenate([im.reshape(-1, 3) for im in ims])).cuda()
    tgt = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in tgs])).cuda()
    grad = torch.empty_like(img)
    loss = torch.zeros(1, device="cuda")
    ws = torch.empty(cgs.loss_recon_workspace_bytes(hw), dtype=torch.uint8, device="cuda")
    render.loss_recon(img, tgt, hw, lam, grad, loss, ws)
    torch.cuda.synchronize()
    go = np.concatenate([g.reshape(-1, 3) for g in grads_o])
    e_loss = abs(loss.item() - loss_o) / max(1.0, abs(loss_o))
    e_grad = rel_l2(grad.cpu().numpy(), go)
    say(f"  loss {loss.item():.7f} vs {loss_o:.7f} (rel {e_loss:.1e}), grad rel L2 {e_grad:.1e}")
    assert e_loss <= LOSS_TOL and e_grad <= GRAD_TOL
    if lam == 0.0:      # pure L1: the same bits as the L1 kernel
        g1 = torch.empty_like(img)
        l1 = torch.zeros(1, device="cuda")
        ws1 = torch.empty(cgs.loss_l1_workspace_bytes(img.numel()), dtype=torch.uint8, device="cuda")
        render.loss_l1(img, tgt, g1, l1, ws1)
        torch.cuda.synchronize()
        assert torch.equal(g1, grad)


def _delta_errors(name, before, after, oracle_after):
    d_gpu = after.astype(np.float64) - before.astype(np.float64)
    d_ora = oracle_after - before.astype(np.float64)
    e = rel_l2(d_gpu, d_ora)
    say(f"  {name}: rel L2 of the update {e:.2e}")
    return e


EPS = {"noise": (1e-4, 1e-3, 1e-3, 1e-3), "drift": (1e6, 1e7, 1e7, 1e7)}


@pytest.mark.parametrize("regime", ["noise", "drift"])
@pytest.mark.parametrize("kind", ["clusters20k_d3", "clusters20k_d3_bf16"])
def test_backward_sgld_fused_layout(kind, regime):
    """Fused codebook: FP32 updated in place, or BF16 with an FP32 master whose
    update refreshes the BF16 rows the renderer reads."""
    wl = small_workload(kind)
    eps = EPS[regime]
    seed, step = 0xC0FFEE1234, 5
    say(f"[sgld] {kind} {regime} eps={eps}")
    r = gpu_renderer(wl)
    pix = [full_pixels(c) for c in wl.cameras]
    base = oracle_render(wl, pix)
    gcols, gfull = oracle_grad_image(wl, pix, base)
    ogm, ogcb = oracle_scene_grads(wl, oracle_render(wl, pix, gcols))
    ds = r.scenes[0]
    gfull_t = torch.from_numpy(gfull).cuda()
    r.forward()
    gm, gcb = r.backward(gfull_t)
    gm_plain, gcb_plain = gm[0].clone(), gcb[0].clone()
    master = ds.cb.float().clone()          # exact: BF16 values widen to FP32 exactly
    means0, cb0 = ds.means.cpu().numpy().copy(), master.cpu().numpy().copy()
    sg = cgs.Sgld(*eps, seed, step, 0)
    r.backward_sgld(gfull_t, sg, [render.sgld_params(ds, master_sr=None if ds.cb.dtype == torch.float32 else master)])
    torch.cuda.synchronize()
    assert torch.equal(r.grad_means[0], gm_plain) and torch.equal(r.grad_cb[0], gcb_plain)
    s = wl.scenes[0]
    K, R = s.cb.shape
    o_cb = otrain.sgld(cb0, ogcb[0], otrain.row_eps(0, R, eps[2], eps[1], eps[3])[None, :],
                       otrain.codebook_noise(K, 0, R, 0, step, seed))
    o_means = otrain.sgld(means0, ogm[0], eps[0], otrain.gaussian_noise(s.n, 0, step, seed)[:, :3])
    new_cb = (ds.cb if ds.cb.dtype == torch.float32 else master).cpu().numpy()
    errs = [_delta_errors("means", means0, ds.means.cpu().numpy(), o_means)]
    for blk, sl in (("ls+q", slice(0, 7)), ("logit", slice(7, 8)), ("sh", slice(8, None))):
        errs.append(_delta_errors(blk, cb0[:, sl], new_cb[:, sl], o_cb[:, sl]))
    assert max(errs) <= GRAD_TOL
    if ds.cb.dtype == torch.bfloat16:        # the renderer's copy is RNE(master)
        want = sc.f32_to_bf16_bits(master.cpu().numpy())
        assert np.array_equal(ds.cb.view(torch.int16).cpu().numpy().view(np.uint16), want)


@pytest.mark.parametrize("bf16", [False, True])
def test_backward_sgld_two_codebooks(bf16):
    """The paper's state (SR and SH codebooks, per-Gaussian opacity): every
    parameter kind takes its own step size and noise stream."""
    say(f"[sgld two codebooks] bf16={bf16}")
    rng = np.random.default_rng(191 + int(bf16))
    n, ksr, ksh, d = 12000, 250, 600, 3
    W, H = 144, 112
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
    cam = sc.pinhole(W, H, (0.2, 0.1, -3.0))
    target = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    rows = np.concatenate([sr32[g2sr], logit[:, None], sh32[g2sh]], 1).astype(np.float32)
    host = sc.Scene(means, np.zeros(n, np.int32), np.zeros((1, 56), np.float32), d)
    pix = full_pixels(cam)
    base = oracle.render_view(host, cam, pix, rows32=rows)
    _, g = oracle.loss_l1(base["color"].reshape(H, W, 3), target)
    g = g.reshape(-1, 3)
    g[base["ambiguous"]] = 0.0
    g32 = g.astype(np.float32)
    og = oracle.render_view(host, cam, pix, grad_color=g32.astype(np.float64), rows32=rows)
    o_sr = oracle.codebook_grad_reduce(og["grad_rows"][:, :7], g2sr, ksr)
    o_sh = oracle.codebook_grad_reduce(og["grad_rows"][:, 8:], g2sh, ksh)
    o_op = og["grad_rows"][:, 7]

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if bf16:
        dsr = dev(sr_bits.view(np.int16)).view(torch.bfloat16)
        dsh = dev(sh_bits.view(np.int16)).view(torch.bfloat16)
    else:
        dsr, dsh = dev(sr32), dev(sh32)
    ds = render.DeviceScene2(dev(means), dev(g2sr), dev(g2sh), dsr, dsh, dev(logit), d)
    r = render.Renderer([ds], [cam], [0])
    r.fit_capacity()
    r.forward()
    m_sr, m_sh = dev(sr32), dev(sh32)         # FP32 masters (used when the codebooks are BF16)
    eps = (2e-4, 3e-3, 1e-3, 5e-4)
    seed, step = 99, 12
    sg = cgs.Sgld(*eps, seed, step, 0)
    r.backward_sgld(dev(g32), sg, [render.sgld_params(ds, master_sr=m_sr, master_sh=m_sh)])
    torch.cuda.synchronize()
    new_sr = (m_sr if bf16 else ds.sr).cpu().numpy()
    new_sh = (m_sh if bf16 else ds.sh).cpu().numpy()
    zg = otrain.gaussian_noise(n, 0, step, seed)
    errs = [_delta_errors("means", means, ds.means.cpu().numpy(), otrain.sgld(means, og["grad_means"], eps[0], zg[:, :3])),
            _delta_errors("opacity", logit, ds.opacity_logit.cpu().numpy(), otrain.sgld(logit, o_op, eps[1], zg[:, 3])),
            _delta_errors("sr", sr32, new_sr, otrain.sgld(sr32, o_sr, eps[2], otrain.codebook_noise(ksr, 0, 7, 0, step, seed))),
            _delta_errors("sh", sh32, new_sh, otrain.sgld(sh32, o_sh, eps[3], otrain.codebook_noise(ksh, 8, 48, 0, step, seed)))]
    assert max(errs) <= GRAD_TOL
    if bf16:
        assert np.array_equal(ds.sr.view(torch.int16).cpu().numpy().view(np.uint16), sc.f32_to_bf16_bits(new_sr))
        assert np.array_equal(ds.sh.view(torch.int16).cpu().numpy().view(np.uint16), sc.f32_to_bf16_bits(new_sh))
