"""ctypes binding of libcgs (include/cgs.h).  Argument marshalling only: every
step of the render runs in the HIP library.  Loading fails loudly when the
library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcgs.so")

CGS_OK, CGS_EINVAL, CGS_EUNSUPPORTED, CGS_ECAPACITY, CGS_EHIP, CGS_EWORKSPACE, CGS_ELIMIT = 0, -1, -2, -3, -4, -5, -6
CGS_F32, CGS_BF16 = 0, 1
MAX_VIEWS = MAX_SCENES = 64

EXPORTS = ("cgs_workspace_bytes", "cgs_render_forward", "cgs_render_backward",
           "cgs_codebook_grad_reduce_workspace_bytes", "cgs_codebook_grad_reduce",
           "cgs_bin_tiles_workspace_bytes", "cgs_bin_tiles", "cgs_loss_l1_workspace_bytes",
           "cgs_loss_l1", "cgs_workspace_layout", "cgs_status_str", "cgs_version", "cgs_sort_stalls",
           "cgs_render_backward_sgld", "cgs_sgld_normals", "cgs_loss_recon_workspace_bytes", "cgs_loss_recon",
           "cgs_mh_workspace_bytes", "cgs_mh_split", "cgs_mh_merge", "cgs_mh_transition",
           "cgs_codebook_grad_reduce_noalloc")


class Camera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("Rt", c_float * 12), ("campos", c_float * 3),
                ("bg", c_float * 3)]


class CbView(ctypes.Structure):
    _fields_ = [("ptr", c_void_p), ("dtype", c_int32), ("row_stride", c_int32), ("rows", c_int64),
                ("col0", c_int32), ("pad_", c_int32)]


class Scene(ctypes.Structure):
    _fields_ = [("n", c_int64), ("sh_degree", c_int32), ("opacity_mode", c_int32),
                ("means", c_void_p), ("idx_sr", c_void_p), ("idx_sh", c_void_p),
                ("sr", CbView), ("sh", CbView), ("opacity_logit", c_void_p)]


class SceneGrads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("sr", c_void_p), ("sr_stride", c_int32), ("sr_col0", c_int32),
                ("sh", c_void_p), ("sh_stride", c_int32), ("sh_col0", c_int32), ("opacity", c_void_p)]


STAGE_EVENTS = 8


class Schedule(ctypes.Structure):
    _fields_ = [("blend_waves_per_block", c_int32), ("tile_order", c_int32), ("persistent", c_int32),
                ("reserved", c_int32),
                ("stage_events", POINTER(c_void_p)), ("n_blend", c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("scenes", POINTER(Scene)), ("n_scenes", c_int32), ("n_views", c_int32),
                ("cameras", POINTER(Camera)), ("view_scene", POINTER(c_int32)),
                ("instance_capacity", c_int64), ("schedule", POINTER(Schedule))]


class WsLayout(ctypes.Structure):
    _fields_ = [("records", c_size_t),
                ("depth_key", c_size_t), ("tile_rect", c_size_t), ("inst_rec", c_size_t),
                ("tile_range", c_size_t), ("n_records", c_int64), ("n_tiles", c_int64)]


class Sgld(ctypes.Structure):
    _fields_ = [("eps_means", ctypes.c_float), ("eps_opacity", ctypes.c_float), ("eps_sr", ctypes.c_float),
                ("eps_sh", ctypes.c_float), ("seed", ctypes.c_uint64), ("step", ctypes.c_uint32),
                ("pad_", ctypes.c_uint32)]


class SceneParams(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("opacity_logit", c_void_p),
                ("sr", c_void_p), ("sr_stride", c_int32), ("sr_col0", c_int32),
                ("sh", c_void_p), ("sh_stride", c_int32), ("sh_col0", c_int32)]


class Mh(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_float), ("eps_split", ctypes.c_float), ("eps_merge", ctypes.c_float),
                ("n_proposals", c_int32), ("seed", ctypes.c_uint64), ("step", ctypes.c_uint32),
                ("pad_", ctypes.c_uint32)]


class MhCodebook(ctypes.Structure):
    _fields_ = [("rows", c_void_p), ("ld", c_int64), ("D", c_int64), ("K_max", c_int64), ("d_rows", c_void_p),
                ("idx", c_void_p), ("n", c_int64), ("mirror", c_void_p), ("mirror_ld", c_int64)]


_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcgs.so; raises if it is missing (build it with build.py)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"libcgs not built: {path} is missing (run paper_2509_03775_amd/build.py)")
    # torch ships its own HIP runtime: load it first so that libcgs binds to
    # the same runtime (and device context) as the tensors it is given
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    pb = POINTER(Batch)
    L.cgs_workspace_bytes.argtypes = [pb]
    L.cgs_workspace_bytes.restype = c_size_t
    L.cgs_render_forward.argtypes = [pb, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]
    L.cgs_render_forward.restype = c_int32
    L.cgs_render_backward.argtypes = [pb, c_void_p, c_void_p, c_void_p, POINTER(SceneGrads), c_void_p, c_size_t,
                                      c_void_p, c_void_p]
    L.cgs_render_backward.restype = c_int32
    L.cgs_codebook_grad_reduce_workspace_bytes.argtypes = [c_int64, c_int64, c_int32]
    L.cgs_codebook_grad_reduce_workspace_bytes.restype = c_size_t
    L.cgs_codebook_grad_reduce.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_int64, c_int32,
                                           c_void_p, c_int64, c_void_p, c_size_t, c_void_p]
    L.cgs_codebook_grad_reduce.restype = c_int32
    L.cgs_codebook_grad_reduce_noalloc.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_int64, c_int32,
                                                   c_void_p, c_int64, c_void_p]
    L.cgs_codebook_grad_reduce_noalloc.restype = c_int32
    L.cgs_bin_tiles_workspace_bytes.argtypes = [c_int64, c_int32, c_int32, c_int32, c_int64]
    L.cgs_bin_tiles_workspace_bytes.restype = c_size_t
    L.cgs_bin_tiles.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_int32, c_int32, c_void_p,
                                c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]
    L.cgs_bin_tiles.restype = c_int32
    L.cgs_loss_l1_workspace_bytes.argtypes = [c_int64]
    L.cgs_loss_l1_workspace_bytes.restype = c_size_t
    L.cgs_loss_l1.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.cgs_loss_l1.restype = c_int32
    L.cgs_render_backward_sgld.argtypes = [pb, c_void_p, c_void_p, c_void_p, POINTER(SceneGrads), POINTER(Sgld),
                                           POINTER(SceneParams), c_void_p, c_size_t, c_void_p, c_void_p]
    L.cgs_render_backward_sgld.restype = c_int32
    L.cgs_sgld_normals.argtypes = [c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                   c_void_p, c_void_p, c_void_p]
    L.cgs_sgld_normals.restype = c_int32
    L.cgs_loss_recon_workspace_bytes.argtypes = [c_int32, POINTER(c_int32)]
    L.cgs_loss_recon_workspace_bytes.restype = c_size_t
    L.cgs_loss_recon.argtypes = [c_void_p, c_void_p, c_int32, POINTER(c_int32), ctypes.c_float, c_void_p, c_void_p,
                                 c_void_p, c_size_t, c_void_p]
    L.cgs_loss_recon.restype = c_int32
    L.cgs_mh_workspace_bytes.argtypes = [POINTER(MhCodebook), c_int32]
    L.cgs_mh_workspace_bytes.restype = c_size_t
    for fn in (L.cgs_mh_split, L.cgs_mh_merge):
        fn.argtypes = [POINTER(MhCodebook), POINTER(Mh), c_void_p, c_size_t, c_void_p]
        fn.restype = c_int32
    L.cgs_mh_transition.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    L.cgs_mh_transition.restype = c_int32
    L.cgs_workspace_layout.argtypes = [pb, POINTER(WsLayout)]
    L.cgs_workspace_layout.restype = c_int32
    L.cgs_status_str.argtypes = [c_int32]
    L.cgs_status_str.restype = ctypes.c_char_p
    L.cgs_version.argtypes = []
    L.cgs_version.restype = c_int32
    L.cgs_sort_stalls.argtypes = []
    L.cgs_sort_stalls.restype = ctypes.c_uint32
    _LIB = L
    return L


class CgsError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = load().cgs_status_str(status).decode()
        super().__init__(f"{fn} failed: {msg} ({status})")
        self.status = status


def check(fn: str, status: int) -> None:
    if status != CGS_OK:
        raise CgsError(fn, status)


def ptr(t) -> int | None:
    """Device (or host) address of a tensor, None for None."""
    return None if t is None else t.data_ptr()


# --- thin wrappers with the C names (pointers are raw integers) -------------

def workspace_bytes(batch: Batch) -> int:
    return load().cgs_workspace_bytes(ctypes.byref(batch))


def render_forward(batch: Batch, image, T_final, n_last, ws, ws_bytes, d_info, stream) -> None:
    check("cgs_render_forward", load().cgs_render_forward(ctypes.byref(batch), image, T_final, n_last, ws,
                                                          ws_bytes, d_info, stream))


def render_backward(batch: Batch, grad_image, T_final, n_last, grads, ws, ws_bytes, d_info, stream) -> None:
    check("cgs_render_backward", load().cgs_render_backward(ctypes.byref(batch), grad_image, T_final, n_last,
                                                            grads, ws, ws_bytes, d_info, stream))


def codebook_grad_reduce_workspace_bytes(n: int, k: int, d: int) -> int:
    return load().cgs_codebook_grad_reduce_workspace_bytes(n, k, d)


def codebook_grad_reduce(g, ld, idx, perm, n, k, d, grad_cb, ld_out, ws, ws_bytes, stream) -> None:
    check("cgs_codebook_grad_reduce", load().cgs_codebook_grad_reduce(g, ld, idx, perm, n, k, d, grad_cb, ld_out,
                                                                      ws, ws_bytes, stream))


def codebook_grad_reduce_noalloc(g, ld, idx, perm, n, k, d, grad_cb, ld_out, stream) -> None:
    check("cgs_codebook_grad_reduce_noalloc",
          load().cgs_codebook_grad_reduce_noalloc(g, ld, idx, perm, n, k, d, grad_cb, ld_out, stream))


def bin_tiles_workspace_bytes(n, tiles_x, tiles_y, n_views, capacity) -> int:
    return load().cgs_bin_tiles_workspace_bytes(n, tiles_x, tiles_y, n_views, capacity)


def bin_tiles(depth_key, trect, view_of, n, tiles_x, tiles_y, n_views, sorted_key, sorted_gid, tile_range,
              capacity, d_info, ws, ws_bytes, stream) -> None:
    check("cgs_bin_tiles", load().cgs_bin_tiles(depth_key, trect, view_of, n, tiles_x, tiles_y, n_views,
                                                sorted_key, sorted_gid, tile_range, capacity, d_info, ws,
                                                ws_bytes, stream))


def loss_l1_workspace_bytes(n: int) -> int:
    return load().cgs_loss_l1_workspace_bytes(n)


def loss_l1(image, target, n, grad, loss, ws, ws_bytes, stream) -> None:
    check("cgs_loss_l1", load().cgs_loss_l1(image, target, n, grad, loss, ws, ws_bytes, stream))


def render_backward_sgld(batch: Batch, grad_image, T_final, n_last, grads, sgld: Sgld, params, ws, ws_bytes,
                         d_info, stream) -> None:
    check("cgs_render_backward_sgld", load().cgs_render_backward_sgld(ctypes.byref(batch), grad_image, T_final,
                                                                      n_last, grads, ctypes.byref(sgld), params, ws,
                                                                      ws_bytes, d_info, stream))


def sgld_normals(n, index0, tag, step, seed, z, words, stream) -> None:
    check("cgs_sgld_normals", load().cgs_sgld_normals(n, index0, tag, step, seed, z, words, stream))


def _hw_array(hw):
    flat = [int(v) for pair in hw for v in pair]
    return (c_int32 * len(flat))(*flat)


def loss_recon_workspace_bytes(hw) -> int:
    return load().cgs_loss_recon_workspace_bytes(len(hw), _hw_array(hw))


def loss_recon(image, target, hw, lambda_ssim, grad, loss, ws, ws_bytes, stream) -> None:
    check("cgs_loss_recon", load().cgs_loss_recon(image, target, len(hw), _hw_array(hw), lambda_ssim, grad, loss,
                                                  ws, ws_bytes, stream))


def mh_workspace_bytes(cb: MhCodebook, n_proposals: int) -> int:
    return load().cgs_mh_workspace_bytes(ctypes.byref(cb), n_proposals)


def mh_split(cb: MhCodebook, p: Mh, ws, ws_bytes, stream) -> None:
    check("cgs_mh_split", load().cgs_mh_split(ctypes.byref(cb), ctypes.byref(p), ws, ws_bytes, stream))


def mh_merge(cb: MhCodebook, p: Mh, ws, ws_bytes, stream) -> None:
    check("cgs_mh_merge", load().cgs_mh_merge(ctypes.byref(cb), ctypes.byref(p), ws, ws_bytes, stream))


def mh_transition(seed: int, step: int) -> int:
    return load().cgs_mh_transition(seed, step)


def workspace_layout(batch: Batch) -> WsLayout:
    out = WsLayout()
    check("cgs_workspace_layout", load().cgs_workspace_layout(ctypes.byref(batch), ctypes.byref(out)))
    return out
