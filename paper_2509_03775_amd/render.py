"""Torch-facing wrapper of libcgs: device-resident scenes, a view batch with its
workspace, and a torch.autograd.Function whose backward calls
cgs_render_backward.  PyTorch supplies device memory and streams only; every
step of the render runs in the HIP library (see cgs.py).
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import cgs
from . import scenes as sc


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class DeviceScene:
    """One scene's state on the GPU in the fused single-codebook layout:
    means float32 [N,3], idx int32 [N], codebook [K, 8 + 3(d+1)^2] in float32
    or bfloat16 (row: log-scale 3, quaternion 4, opacity logit 1, SH).  The
    codebook may be a row-strided view (rows padded for alignment)."""

    def __init__(self, means: torch.Tensor, idx: torch.Tensor, cb: torch.Tensor, sh_degree: int):
        assert means.dtype == torch.float32 and means.is_contiguous() and means.dim() == 2 and means.shape[1] == 3
        assert idx.dtype == torch.int32 and idx.is_contiguous() and idx.shape[0] == means.shape[0]
        assert cb.dtype in (torch.float32, torch.bfloat16) and cb.dim() == 2 and cb.stride(1) == 1
        assert cb.shape[1] == sc.row_width(sh_degree) and cb.stride(0) >= cb.shape[1]
        self.means, self.idx, self.cb, self.sh_degree = means, idx, cb, sh_degree

    @classmethod
    def from_host(cls, s: sc.Scene, device="cuda", bf16: Optional[bool] = None) -> "DeviceScene":
        use_bf16 = (s.cb_bf16 is not None) if bf16 is None else bf16
        means = torch.from_numpy(np.ascontiguousarray(s.means)).to(device)
        idx = torch.from_numpy(np.ascontiguousarray(s.idx)).to(device)
        if use_bf16:
            bits = s.cb_bf16 if s.cb_bf16 is not None else sc.f32_to_bf16_bits(s.cb)
            cb = torch.from_numpy(bits.view(np.int16)).to(device).view(torch.bfloat16)
        else:
            cb = torch.from_numpy(np.ascontiguousarray(s.cb)).to(device)
        # rows padded to whole 128-byte lines: a Gaussian's row gather then
        # touches one or two lines, never a line shared with the next row
        k, r = cb.shape
        line = 128 // cb.element_size()
        store = torch.zeros((k, (r + line - 1) // line * line), dtype=cb.dtype, device=device)
        store[:, :r] = cb
        return cls(means, idx, store[:, :r], s.sh_degree)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def k(self) -> int:
        return int(self.cb.shape[0])

    @property
    def r(self) -> int:
        return int(self.cb.shape[1])

    def descriptor(self) -> cgs.Scene:
        dt = cgs.CGS_BF16 if self.cb.dtype == torch.bfloat16 else cgs.CGS_F32
        d = cgs.Scene()
        d.n = self.n
        d.sh_degree = self.sh_degree
        d.opacity_mode = 1
        d.means = self.means.data_ptr()
        d.idx_sr = self.idx.data_ptr()
        d.idx_sh = self.idx.data_ptr()
        d.sr = cgs.CbView(self.cb.data_ptr(), dt, self.cb.stride(0), self.k, 0, 0)
        d.sh = cgs.CbView(self.cb.data_ptr(), dt, self.cb.stride(0), self.k, 8, 0)
        d.opacity_logit = None
        return d


class DeviceScene2:
    """The paper's state layout (Sec. 4.1, Fig. 4) on the GPU: an SR codebook
    [|SR|, 7] (log-scale 3, quaternion 4), an SH codebook [|SH|, 3(d+1)^2], two
    index arrays g2sr / g2sh and a per-Gaussian opacity logit."""

    def __init__(self, means, idx_sr, idx_sh, sr, sh, opacity_logit, sh_degree: int):
        assert means.dtype == torch.float32 and means.is_contiguous() and means.shape[1] == 3
        for t in (idx_sr, idx_sh):
            assert t.dtype == torch.int32 and t.is_contiguous() and t.shape[0] == means.shape[0]
        assert sr.dtype == sh.dtype and sr.dtype in (torch.float32, torch.bfloat16)
        assert sr.shape[1] == 7 and sh.shape[1] == 3 * (sh_degree + 1) ** 2
        assert opacity_logit.dtype == torch.float32 and opacity_logit.shape[0] == means.shape[0]
        self.means, self.idx_sr, self.idx_sh = means, idx_sr, idx_sh
        self.sr, self.sh, self.opacity_logit, self.sh_degree = sr.contiguous(), sh.contiguous(), opacity_logit, sh_degree

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def descriptor(self) -> cgs.Scene:
        dt = cgs.CGS_BF16 if self.sr.dtype == torch.bfloat16 else cgs.CGS_F32
        d = cgs.Scene()
        d.n = self.n
        d.sh_degree = self.sh_degree
        d.opacity_mode = 0
        d.means = self.means.data_ptr()
        d.idx_sr = self.idx_sr.data_ptr()
        d.idx_sh = self.idx_sh.data_ptr()
        d.sr = cgs.CbView(self.sr.data_ptr(), dt, 7, int(self.sr.shape[0]), 0, 0)
        d.sh = cgs.CbView(self.sh.data_ptr(), dt, int(self.sh.shape[1]), int(self.sh.shape[0]), 0, 0)
        d.opacity_logit = self.opacity_logit.data_ptr()
        return d

    def grad_buffers(self, device):
        return (torch.empty_like(self.means),
                torch.empty((self.sr.shape[0], 7), dtype=torch.float32, device=device),
                torch.empty((self.sh.shape[0], self.sh.shape[1]), dtype=torch.float32, device=device),
                torch.empty(self.n, dtype=torch.float32, device=device))


def camera_struct(c: sc.Camera) -> cgs.Camera:
    out = cgs.Camera()
    out.width, out.height = int(c.width), int(c.height)
    out.fx, out.fy, out.cx, out.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
    out.Rt[:] = [float(x) for x in np.asarray(c.Rt, np.float32).reshape(12)]
    out.campos[:] = [float(x) for x in np.asarray(c.campos, np.float32)]
    out.bg[:] = [float(x) for x in np.asarray(c.bg, np.float32)]
    return out


class Renderer:
    """A batch of views over device scenes with a persistent workspace and
    preallocated outputs.  forward()/backward() enqueue on the current stream
    and never synchronise (graph-capturable); fit_capacity() sizes the
    instance buffers from a measured run."""

    def __init__(self, scenes: Sequence[DeviceScene], cameras: Sequence[sc.Camera],
                 view_scene: Sequence[int], capacity: Optional[int] = None,
                 waves_per_block: int = 1, tile_order: int = 0, device="cuda", persistent: int = 0):
        self.scenes = list(scenes)
        self.cameras = list(cameras)
        self.device = torch.device(device)
        nv, ns = len(self.cameras), len(self.scenes)
        self._scene_arr = (cgs.Scene * ns)(*[s.descriptor() for s in self.scenes])
        self._cam_arr = (cgs.Camera * nv)(*[camera_struct(c) for c in self.cameras])
        self._vs_arr = (ctypes.c_int32 * nv)(*[int(v) for v in view_scene])
        self.view_scene = [int(v) for v in view_scene]
        self._sched = cgs.Schedule()
        self._sched.blend_waves_per_block = waves_per_block
        self._sched.tile_order = tile_order
        self._sched.persistent = persistent
        self.n_pixels = sum(c.width * c.height for c in self.cameras)
        self.pix_off = np.concatenate([[0], np.cumsum([c.width * c.height for c in self.cameras])]).astype(np.int64)
        if capacity is None:
            capacity = max(1024, int(3 * sum(self.scenes[v].n for v in self.view_scene)))
        self.batch = cgs.Batch()
        self.batch.scenes = ctypes.cast(self._scene_arr, ctypes.POINTER(cgs.Scene))
        self.batch.n_scenes = ns
        self.batch.n_views = nv
        self.batch.cameras = ctypes.cast(self._cam_arr, ctypes.POINTER(cgs.Camera))
        self.batch.view_scene = ctypes.cast(self._vs_arr, ctypes.POINTER(ctypes.c_int32))
        self.batch.schedule = ctypes.pointer(self._sched)
        self.image = torch.empty((self.n_pixels, 3), dtype=torch.float32, device=self.device)
        self.T_final = torch.empty(self.n_pixels, dtype=torch.float32, device=self.device)
        self.n_last = torch.empty(self.n_pixels, dtype=torch.int32, device=self.device)
        self.d_info = torch.zeros(4, dtype=torch.int64, device=self.device)
        # forward() calls so far: the backward reads the binning, T_final and
        # n_last the last forward left in the workspace, so a differentiable
        # render checks that no other forward ran in between
        self.generation = 0
        self.grad_means, self.grad_cb, self.grad_sr, self.grad_sh, self.grad_opacity = [], [], [], [], []
        gr = []
        for s in self.scenes:
            g = cgs.SceneGrads()
            if isinstance(s, DeviceScene2):
                gm, gsr, gsh, gop = s.grad_buffers(self.device)
                g.means = gm.data_ptr()
                g.sr, g.sr_stride, g.sr_col0 = gsr.data_ptr(), 7, 0
                g.sh, g.sh_stride, g.sh_col0 = gsh.data_ptr(), int(gsh.shape[1]), 0
                g.opacity = gop.data_ptr()
                self.grad_means.append(gm)
                self.grad_cb.append(None)
                self.grad_sr.append(gsr)
                self.grad_sh.append(gsh)
                self.grad_opacity.append(gop)
            else:
                gm = torch.empty_like(s.means)
                gc = torch.empty((s.k, s.r), dtype=torch.float32, device=self.device)
                g.means = gm.data_ptr()
                g.sr, g.sr_stride, g.sr_col0 = gc.data_ptr(), s.r, 0
                g.sh, g.sh_stride, g.sh_col0 = gc.data_ptr(), s.r, 8
                g.opacity = None
                self.grad_means.append(gm)
                self.grad_cb.append(gc)
                self.grad_sr.append(None)
                self.grad_sh.append(None)
                self.grad_opacity.append(None)
            gr.append(g)
        self._grads = (cgs.SceneGrads * ns)(*gr)
        self.set_capacity(capacity)

    def set_schedule(self, waves_per_block: int, tile_order: int, persistent: int = 0) -> None:
        """Change the blend launch schedule (issue order only; results are
        bitwise unchanged)."""
        self._sched.blend_waves_per_block = int(waves_per_block)
        self._sched.tile_order = int(tile_order)
        self._sched.persistent = int(persistent)

    @property
    def schedule(self):
        return (int(self._sched.blend_waves_per_block or 1), int(self._sched.tile_order),
                int(self._sched.persistent))

    def set_capacity(self, capacity: int) -> None:
        self.capacity = int(capacity)
        self.batch.instance_capacity = self.capacity
        nbytes = cgs.workspace_bytes(self.batch)
        if nbytes == 0:
            raise cgs.CgsError("cgs_workspace_bytes", cgs.CGS_EINVAL)
        self.ws_bytes = nbytes
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def forward(self, stream=None) -> torch.Tensor:
        self.generation += 1
        cgs.render_forward(self.batch, self.image.data_ptr(), self.T_final.data_ptr(), self.n_last.data_ptr(),
                           self.ws.data_ptr(), self.ws_bytes, self.d_info.data_ptr(), _stream_ptr(stream))
        return self.image

    def backward(self, grad_image: torch.Tensor, stream=None):
        assert grad_image.dtype == torch.float32 and grad_image.is_contiguous()
        assert grad_image.numel() == 3 * self.n_pixels
        cgs.render_backward(self.batch, grad_image.data_ptr(), self.T_final.data_ptr(), self.n_last.data_ptr(),
                            self._grads, self.ws.data_ptr(), self.ws_bytes, self.d_info.data_ptr(),
                            _stream_ptr(stream))
        return self.grad_means, self.grad_cb

    def backward_sgld(self, grad_image: torch.Tensor, sgld: "cgs.Sgld", params: Sequence["cgs.SceneParams"],
                      stream=None):
        """backward() plus one fused SGLD step of every parameter (params:
        one cgs.SceneParams per scene, e.g. from sgld_params())."""
        assert grad_image.dtype == torch.float32 and grad_image.is_contiguous()
        assert grad_image.numel() == 3 * self.n_pixels and len(params) == len(self.scenes)
        arr = (cgs.SceneParams * len(params))(*params)
        cgs.render_backward_sgld(self.batch, grad_image.data_ptr(), self.T_final.data_ptr(), self.n_last.data_ptr(),
                                 self._grads, sgld, arr, self.ws.data_ptr(), self.ws_bytes, self.d_info.data_ptr(),
                                 _stream_ptr(stream))
        return self.grad_means, self.grad_cb

    def instances(self) -> int:
        """Instances the last forward needed (synchronises)."""
        return int(self.d_info[1].item())

    def fit_capacity(self, slack: float = 1.05) -> int:
        """Run the forward, and if the instance buffers overflowed, grow them
        and run again (synchronises; call outside timed or captured regions)."""
        self.forward()
        torch.cuda.synchronize()
        info = self.d_info.cpu().numpy()
        if info[0] == cgs.CGS_ECAPACITY:
            self.set_capacity(int(info[1] * slack) + 1024)
            self.forward()
            torch.cuda.synchronize()
            info = self.d_info.cpu().numpy()
            if info[0] != cgs.CGS_OK:
                raise cgs.CgsError("cgs_render_forward (capacity)", int(info[0]))
        return int(info[1])

    def layout(self) -> cgs.WsLayout:
        return cgs.workspace_layout(self.batch)

    def view_image(self, v: int) -> torch.Tensor:
        c = self.cameras[v]
        return self.image[self.pix_off[v]:self.pix_off[v + 1]].view(c.height, c.width, 3)


class CgsRenderFunction(torch.autograd.Function):
    """image = render(means_0, codebook_0, means_1, codebook_1, ...).

    The backward recomputes each blended Gaussian's transmittance from the
    per-pixel final transmittance instead of storing it per pair.  It reads
    what the forward left in the renderer (binning, T_final, n_last), so it
    raises if the renderer ran another forward since, and the inputs are saved
    for backward so that autograd raises if one was modified in place."""

    @staticmethod
    def forward(ctx, renderer: Renderer, *tensors):
        ctx.renderer = renderer
        img = renderer.forward()
        ctx.generation = renderer.generation
        ctx.save_for_backward(*tensors)
        return img.clone()

    @staticmethod
    def backward(ctx, grad_image):
        r: Renderer = ctx.renderer
        ctx.saved_tensors      # autograd's in-place modification check
        if r.generation != ctx.generation:
            raise RuntimeError("render backward: the renderer ran another forward after this one, so the "
                               "binning and transmittance this backward needs are gone; call render() again")
        gm, gc = r.backward(grad_image.contiguous().float())
        out: List[Optional[torch.Tensor]] = [None]
        for s, m, c in zip(r.scenes, gm, gc):
            out.append(m.clone())
            out.append(c.clone().to(s.cb.dtype))
        return tuple(out)


def render(renderer: Renderer) -> torch.Tensor:
    """Differentiable render of every view of the batch ([pixels, 3])."""
    tensors = []
    for s in renderer.scenes:
        tensors += [s.means, s.cb]
    return CgsRenderFunction.apply(renderer, *tensors)


def sgld_params(scene, master_sr: Optional[torch.Tensor] = None,
                master_sh: Optional[torch.Tensor] = None) -> "cgs.SceneParams":
    """The FP32 parameters an SGLD step updates for a scene: its own means
    (and per-Gaussian opacity) in place; its codebook(s) in place when FP32,
    else the given FP32 masters (fused layout: master_sr = the [K, R] master,
    master_sh unused)."""
    p = cgs.SceneParams()
    p.means = scene.means.data_ptr()
    if isinstance(scene, DeviceScene2):
        sr = scene.sr if scene.sr.dtype == torch.float32 else master_sr
        sh = scene.sh if scene.sh.dtype == torch.float32 else master_sh
        assert sr is not None and sh is not None and sr.dtype == torch.float32 and sh.dtype == torch.float32
        p.opacity_logit = scene.opacity_logit.data_ptr()
        p.sr, p.sr_stride, p.sr_col0 = sr.data_ptr(), int(sr.shape[1]), 0
        p.sh, p.sh_stride, p.sh_col0 = sh.data_ptr(), int(sh.shape[1]), 0
    else:
        cb = scene.cb if scene.cb.dtype == torch.float32 else master_sr
        assert cb is not None and cb.dtype == torch.float32 and cb.shape == scene.cb.shape and cb.stride(1) == 1
        p.opacity_logit = None
        p.sr, p.sr_stride, p.sr_col0 = cb.data_ptr(), int(cb.stride(0)), 0
        p.sh, p.sh_stride, p.sh_col0 = cb.data_ptr(), int(cb.stride(0)), 8
    return p


class CodebookMoves:
    """A codebook under the Metropolis-Hastings split / merge moves: FP32 rows
    [K_max, ld] (D values from column 0), the live row count on the device,
    the Gaussians' row indices, an optional BF16 copy the renderer reads."""

    def __init__(self, rows: torch.Tensor, n_live: int, idx: torch.Tensor, D: Optional[int] = None,
                 mirror: Optional[torch.Tensor] = None, n_proposals: int = 4096):
        assert rows.dtype == torch.float32 and rows.is_contiguous() and idx.dtype == torch.int32
        self.rows, self.idx, self.mirror = rows, idx, mirror
        self.d_rows = torch.tensor([n_live], dtype=torch.int64, device=rows.device)
        self.cb = cgs.MhCodebook(rows.data_ptr(), int(rows.shape[1]), int(D or rows.shape[1]), int(rows.shape[0]),
                                 self.d_rows.data_ptr(), idx.data_ptr(), int(idx.numel()),
                                 None if mirror is None else mirror.data_ptr(),
                                 0 if mirror is None else int(mirror.shape[1]))
        self.n_proposals = n_proposals
        nb = cgs.mh_workspace_bytes(self.cb, n_proposals)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=rows.device)

    def params(self, lam: float, eps_split: float, eps_merge: float, seed: int, step: int) -> "cgs.Mh":
        return cgs.Mh(lam, eps_split, eps_merge, self.n_proposals, seed, step, 0)

    def split(self, p: "cgs.Mh", stream=None) -> None:
        cgs.mh_split(self.cb, p, self.ws.data_ptr(), self.ws.numel(), _stream_ptr(stream))

    def merge(self, p: "cgs.Mh", stream=None) -> None:
        cgs.mh_merge(self.cb, p, self.ws.data_ptr(), self.ws.numel(), _stream_ptr(stream))

    def live_rows(self) -> int:
        """Live row count (synchronises)."""
        return int(self.d_rows.item())


def loss_recon(image: torch.Tensor, target: torch.Tensor, hw: Sequence[Sequence[int]], lambda_ssim: float,
               grad: torch.Tensor, loss: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    """Eq. 4's (1 - lambda) L1 + lambda (1 - SSIM) and its gradient (writes
    grad and loss); hw = [(height, width)] per view."""
    cgs.loss_recon(image.data_ptr(), target.data_ptr(), hw, float(lambda_ssim), grad.data_ptr(), loss.data_ptr(),
                   ws.data_ptr(), ws.numel(), _stream_ptr(stream))


def loss_l1(image: torch.Tensor, target: torch.Tensor, grad: torch.Tensor, loss: torch.Tensor,
            ws: torch.Tensor, stream=None) -> None:
    """L1 loss and its gradient by the library kernel (writes grad and loss)."""
    n = image.numel()
    cgs.loss_l1(image.data_ptr(), target.data_ptr(), n, grad.data_ptr(), loss.data_ptr(), ws.data_ptr(),
                ws.numel(), _stream_ptr(stream))
