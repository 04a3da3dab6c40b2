"""ORACLE (test infrastructure only): a plain, slow FP64 reference of the
codebook-indexed differentiable Gaussian-splatting render.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does.  It shares no code with the HIP
path: the only common module is the seeded input generator.

What it computes (paper Sec. 2.1 Eq. 1-3 for the render, Sec. 2.2 and
Sec. 4.1 for the codebook state, Sec. 4.4 for the gradient the parameter
update needs):
  * every Gaussian reads its parameters from the codebook row its index names
    (log-scale 3, quaternion 4, opacity logit 1, SH 3(d+1)^2);
  * scale = exp(log-scale), quaternion normalised, opacity = sigmoid(logit);
  * Sigma = R(q) S S^T R(q)^T (Eq. 2), projected to the image by the
    perspective Jacobian J and camera rotation W: Sigma2D = J W Sigma W^T J^T
    + 0.3 I, conic = Sigma2D^-1;
  * view-dependent colour = max(0, sum_lm Y_lm(dir) k_lm + 1/2) with the real
    orthonormal spherical harmonics (Condon-Shortley phase), dir the unit
    vector from the camera centre to the mean;
  * front-to-back compositing (Eq. 3) by brute force per pixel (composite.c);
  * gradients: reverse mode through the compositing (composite.c), then
    PyTorch autograd through the per-Gaussian projection above, then the
    codebook sum G[k] = sum_{i: idx_i = k} dL/dtheta_i.
Discrete decisions (culling, depth order, tile rectangle) come from the FP32
skeleton in keyspec.c; every continuous value is FP64.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

AMBIGUITY_MARGIN = 1e-4


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        L.ok_keyspec.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]
        L.ok_keyspec.restype = None
        L.ok_exp.argtypes = [ctypes.c_float]
        L.ok_exp.restype = ctypes.c_float
        L.oc_composite.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oc_composite.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# FP32 discrete skeleton (keyspec.c)
# --------------------------------------------------------------------------

def cam_f32(cam) -> np.ndarray:
    return np.concatenate([np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float32),
                           np.asarray(cam.Rt, np.float32).reshape(12)]).astype(np.float32)


def keyspec(means: np.ndarray, rows7: np.ndarray, cam):
    """Cull flag, depth key and half-open tile rectangle of each Gaussian."""
    n = means.shape[0]
    means = np.ascontiguousarray(means, np.float32)
    rows7 = np.ascontiguousarray(rows7, np.float32)
    key = np.empty(n, np.uint32)
    trect = np.empty((n, 4), np.uint16)
    kept = np.empty(n, np.uint8)
    c = cam_f32(cam)
    lib().ok_keyspec(n, _p(means), _p(rows7), _p(c), cam.width, cam.height, _p(key), _p(trect), _p(kept))
    return key, trect, kept.astype(bool)


def exp_f32(x: float) -> float:
    return float(lib().ok_exp(ctypes.c_float(x)))


# --------------------------------------------------------------------------
# Real spherical harmonics from their definition
# --------------------------------------------------------------------------

def _sh_terms(lmax: int):
    """For each (l, m): the factor and the power-basis coefficients of
    d^|m| P_l / dz^|m| so that
      Y_lm = f * (d^|m| P_l/dz^|m|)(z) * {Re (x+iy)^m  (m>0); 1 (m=0); Im (x+iy)^|m| (m<0)}
    with f = (-1)^|m| sqrt(2 - delta_m0) sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!).
    This is the real orthonormal basis built from the complex harmonics that
    carry the Condon-Shortley phase; on the unit sphere (1-z^2)^{|m|/2} e^{i|m|phi}
    equals (x+iy)^|m|."""
    out = []
    for l in range(lmax + 1):
        Pl = np.polynomial.legendre.Legendre.basis(l).convert(kind=np.polynomial.Polynomial)
        for m in range(-l, l + 1):
            am = abs(m)
            dP = Pl.deriv(am) if am > 0 else Pl
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            f = (-1) ** am * norm * (math.sqrt(2.0) if m != 0 else 1.0)
            out.append((l, m, f, np.asarray(dP.coef, np.float64)))
    return out


def sh_basis(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Y_j(dir) for j = l*l + l + m, dirs [n,3] unit vectors (float64)."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    cols = []
    for (l, m, f, coef) in _sh_terms(degree):
        poly = torch.zeros_like(z)
        for c in coef[::-1]:
            poly = poly * z + float(c)
        if m > 0:
            ang = re[m]
        elif m < 0:
            ang = im[-m]
        else:
            ang = torch.ones_like(z)
        cols.append(f * poly * ang)
    return torch.stack(cols, dim=1)


# --------------------------------------------------------------------------
# FP64 per-Gaussian projection (differentiable)
# --------------------------------------------------------------------------

def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the unit quaternion (w, x, y, z) (Eq. 2's R(q))."""
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def covariance3d(ls: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    """Sigma = R(q) S S^T R(q)^T with S = diag(exp(ls)), q normalised (Eq. 2)."""
    qn = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    Rm = quat_to_rot(qn)
    M = Rm * torch.exp(ls)[:, None, :]
    return M @ M.transpose(-1, -2)


def project(means: torch.Tensor, rows: torch.Tensor, cam, sh_degree: int) -> Dict[str, torch.Tensor]:
    """Per-Gaussian 2D footprint and colour for one camera (FP64).

    means [n,3], rows [n,R]; returns dict with 'rec' [n,9] = u v A B C o r g b
    and intermediates used by the tests."""
    Rt = torch.tensor(np.asarray(cam.Rt, np.float64).reshape(3, 4), dtype=torch.float64)
    Wr, t = Rt[:, :3], Rt[:, 3]
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    xc = means @ Wr.T + t
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    tx, ty = x / z, y / z
    limx = 1.3 * (0.5 * cam.width / fx)
    limy = 1.3 * (0.5 * cam.height / fy)
    txc = torch.clamp(tx, -limx, limx)
    tyc = torch.clamp(ty, -limy, limy)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * txc / z], -1),
                     torch.stack([zero, fy / z, -fy * tyc / z], -1)], -2)       # [n,2,3]
    Sig = covariance3d(rows[:, 0:3], rows[:, 3:7])
    T = J @ Wr                                                                    # [n,2,3]
    S2 = T @ Sig @ T.transpose(-1, -2) + 0.3 * torch.eye(2, dtype=torch.float64)
    a, b, c = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
    det = a * c - b * b
    A, B, C = c / det, -b / det, a / det
    u = fx * tx + cx
    v = fy * ty + cy
    o = torch.sigmoid(rows[:, 7])
    campos = torch.tensor(np.asarray(cam.campos, np.float64), dtype=torch.float64)
    d = means - campos
    dirs = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    nco = (sh_degree + 1) ** 2
    Y = sh_basis(dirs, sh_degree)                                                 # [n,nco]
    k = rows[:, 8:8 + 3 * nco].reshape(-1, nco, 3)
    col = torch.clamp((Y[:, :, None] * k).sum(1) + 0.5, min=0.0)
    rec = torch.stack([u, v, A, B, C, o, col[:, 0], col[:, 1], col[:, 2]], -1)
    return {"rec": rec, "Sigma3D": Sig, "Sigma2D": S2, "xc": xc}


# --------------------------------------------------------------------------
# Codebook-gradient reduction and tile binning by their definitions
# --------------------------------------------------------------------------

def codebook_grad_reduce(g: np.ndarray, idx: np.ndarray, k: int) -> np.ndarray:
    """G[k] = sum over Gaussians i with idx_i == k of g_i (FP64)."""
    out = np.zeros((k, g.shape[1]), np.float64)
    np.add.at(out, np.asarray(idx, np.int64), np.asarray(g, np.float64))
    return out


def bin_tiles(depth_key: np.ndarray, trect: np.ndarray, view_of: Optional[np.ndarray],
              tiles_x: int, tiles_y: int, n_views: int):
    """Every (Gaussian, overlapped tile) instance keyed by
    (view*tiles + tile) << 32 | depth bits, emitted in Gaussian order (tiles
    row-major), then stably sorted by key.  Returns sorted keys (uint64),
    Gaussian ids (uint32) and per-tile half-open ranges [n_views*tiles, 2]."""
    n = depth_key.shape[0]
    ntile = tiles_x * tiles_y
    keys: List[int] = []
    gids: List[int] = []
    for i in range(n):
        x0, y0, x1, y1 = (int(v) for v in trect[i])
        vw = 0 if view_of is None else int(view_of[i])
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                t = vw * ntile + ty * tiles_x + tx
                keys.append((t << 32) | int(depth_key[i]))
                gids.append(i)
    keys_a = np.asarray(keys, np.uint64)
    gids_a = np.asarray(gids, np.uint32)
    o = np.argsort(keys_a, kind="stable")
    sk, sg = keys_a[o], gids_a[o]
    tiles = (sk >> np.uint64(32)).astype(np.int64)
    allt = np.arange(n_views * ntile + 1)
    bounds = np.searchsorted(tiles, allt, side="left")
    ranges = np.stack([bounds[:-1], bounds[1:]], 1).astype(np.uint32)
    return sk, sg, ranges


def loss_l1(image: np.ndarray, target: np.ndarray):
    """Mean absolute error over every pixel and channel and its gradient
    (Eq. 4 with the SSIM weight set to zero); sign(0) = 0."""
    diff = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    n = diff.size
    return float(np.abs(diff).sum() / n), np.sign(diff) / n


# --------------------------------------------------------------------------
# One view, brute force
# --------------------------------------------------------------------------

def decode_rows(scene) -> np.ndarray:
    """Per-Gaussian codebook rows as the renderer reads them (float32 values;
    BF16 storage decoded exactly)."""
    if scene.cb_bf16 is not None:
        cb = (scene.cb_bf16.astype(np.uint32) << 16).view(np.float32)
    else:
        cb = scene.cb
    return cb[np.asarray(scene.idx, np.int64)]


def tiles_of_pixels(pix: np.ndarray) -> np.ndarray:
    return np.unique((pix[:, 1] >> 4).astype(np.int64) * 100000 + (pix[:, 0] >> 4))


def render_view(scene, cam, pixels: Optional[np.ndarray] = None,
                grad_color: Optional[np.ndarray] = None,
                frozen: Optional[dict] = None, margin: float = AMBIGUITY_MARGIN,
                rows32: Optional[np.ndarray] = None, means32: Optional[np.ndarray] = None,
                want_lists: bool = False, rec_margin: Optional[np.ndarray] = None) -> dict:
    """Render the requested pixels of one view (all pixels if None).

    grad_color [n_pix,3]: dL/dC at those pixels -> returns per-Gaussian
    'grad_means' [N,3] and 'grad_rows' [N,R] (FP64).
    frozen: decisions of an earlier call ({'kept','order','trect','fz_ptr',
    'fz_rec'}), replayed exactly (finite differences with a frozen active set).
    rows32/means32 override the scene's values (perturbed copies).
    rec_margin [N] (optional, per Gaussian): a wider ambiguity margin for
    Gaussians whose FP32 alpha is known to be less accurate; it applies to
    their alpha test and to every transmittance test after them."""
    W, H = cam.width, cam.height
    if pixels is None:
        yy, xx = np.mgrid[0:H, 0:W]
        pixels = np.stack([xx.ravel(), yy.ravel()], 1).astype(np.int32)
    pixels = np.ascontiguousarray(pixels, np.int32)
    npix = pixels.shape[0]
    if rows32 is None:
        rows32 = decode_rows(scene)
    if means32 is None:
        means32 = scene.means
    n = means32.shape[0]

    if frozen is None:
        key, trect, kept = keyspec(means32, rows32[:, :7], cam)
        gid = np.arange(n)
        sel = np.nonzero(kept)[0]
        # Only Gaussians whose rectangle holds a requested tile can matter.
        tset = tiles_of_pixels(pixels)
        if tset.size < (W + 15) // 16 * ((H + 15) // 16):
            tyy, txx = tset // 100000, tset % 100000
            need = np.zeros(sel.size, bool)
            tr = trect[sel].astype(np.int64)
            for a in range(0, tset.size, 64):
                bx, by = txx[a:a + 64], tyy[a:a + 64]
                m = ((tr[:, 0:1] <= bx[None]) & (bx[None] < tr[:, 2:3]) &
                     (tr[:, 1:2] <= by[None]) & (by[None] < tr[:, 3:4]))
                need |= m.any(1)
            sel = sel[need]
        order = sel[np.lexsort((gid[sel], key[sel]))]
        trect_o = np.ascontiguousarray(trect[order].astype(np.int32))
    else:
        order = frozen["order"]
        trect_o = frozen["trect_o"]
        key = frozen.get("key")
        kept = frozen.get("kept")

    want_grad = grad_color is not None
    mt = torch.tensor(np.asarray(means32[order], np.float64), requires_grad=want_grad)
    rt = torch.tensor(np.asarray(rows32[order], np.float64), requires_grad=want_grad)
    with torch.set_grad_enabled(want_grad):
        pr = project(mt, rt, cam, scene.sh_degree)
    rec = np.ascontiguousarray(pr["rec"].detach().numpy(), np.float64)

    color = np.empty((npix, 3), np.float64)
    T = np.empty(npix, np.float64)
    nlast = np.empty(npix, np.int32)
    amb = np.empty(npix, np.int32)
    ncon = np.empty(npix, np.int32)
    bg = np.asarray(cam.bg, np.float64)
    grad_rec = np.zeros_like(rec) if want_grad else None
    gc = np.ascontiguousarray(grad_color, np.float64) if want_grad else None
    L = lib()
    rm = None if rec_margin is None else np.ascontiguousarray(np.asarray(rec_margin, np.float64)[order])
    if frozen is None:
        rc = L.oc_composite(rec.shape[0], _p(rec), _p(trect_o), W, H, _p(bg), npix, _p(pixels),
                            _p(color), _p(T), _p(nlast), _p(amb), _p(ncon), _p(gc), _p(grad_rec),
                            margin, 0, None, None, _p(rm))
        fz_ptr = fz_rec = None
        if want_lists:
            fz_ptr = np.zeros(npix + 1, np.int64)
            fz_ptr[1:] = np.cumsum(ncon)
            fz_rec = np.empty(int(fz_ptr[-1]), np.int64)
            c2, T2, n2, a2, k2 = (np.empty_like(color), np.empty_like(T), np.empty_like(nlast),
                                  np.empty_like(amb), np.empty_like(ncon))
            rc |= L.oc_composite(rec.shape[0], _p(rec), _p(trect_o), W, H, _p(bg), npix, _p(pixels),
                                 _p(c2), _p(T2), _p(n2), _p(a2), _p(k2), None, None,
                                 margin, 0, _p(fz_ptr), _p(fz_rec), _p(rm))
    else:
        fz_ptr, fz_rec = frozen["fz_ptr"], frozen["fz_rec"]
        rc = L.oc_composite(rec.shape[0], _p(rec), _p(trect_o), W, H, _p(bg), npix, _p(pixels),
                            _p(color), _p(T), _p(nlast), _p(amb), _p(ncon), _p(gc), _p(grad_rec),
                            margin, 1, _p(fz_ptr), _p(fz_rec), _p(rm))
    if rc != 0:
        raise MemoryError("oracle compositing ran out of memory")
    out = {"color": color, "T": T, "n_last": nlast, "ambiguous": amb.astype(bool),
           "n_contrib": ncon, "pixels": pixels, "order": order, "n_records": rec.shape[0],
           "key": key, "kept": kept,
           "frozen": {"order": order, "trect_o": trect_o, "fz_ptr": fz_ptr, "fz_rec": fz_rec,
                      "key": key, "kept": kept}}
    if want_grad:
        gm, gr = torch.autograd.grad(pr["rec"], [mt, rt], torch.from_numpy(grad_rec))
        grad_means = np.zeros((n, 3), np.float64)
        grad_rows = np.zeros((n, rows32.shape[1]), np.float64)
        grad_means[order] = gm.numpy()
        grad_rows[order] = gr.numpy()
        out["grad_means"] = grad_means
        out["grad_rows"] = grad_rows
        out["grad_rec"] = grad_rec
    return out


def render_workload(wl, pixels: Optional[Sequence[Optional[np.ndarray]]] = None,
                    grad_colors: Optional[Sequence[Optional[np.ndarray]]] = None) -> List[dict]:
    """Render every view of a workload; with grad_colors also return, per
    scene, the mean gradients and the codebook gradient (views summed)."""
    outs = []
    V = len(wl.cameras)
    acc_m = [np.zeros((s.n, 3)) for s in wl.scenes]
    acc_r = [np.zeros((s.n, s.r)) for s in wl.scenes]
    for v in range(V):
        sc = wl.scenes[int(wl.view_scene[v])]
        px = None if pixels is None else pixels[v]
        gcol = None if grad_colors is None else grad_colors[v]
        o = render_view(sc, wl.cameras[v], px, gcol)
        if gcol is not None:
            acc_m[int(wl.view_scene[v])] += o["grad_means"]
            acc_r[int(wl.view_scene[v])] += o["grad_rows"]
        outs.append(o)
    if grad_colors is not None:
        for s, sc in enumerate(wl.scenes):
            outs.append({"scene": s, "grad_means": acc_m[s],
                         "grad_cb": codebook_grad_reduce(acc_r[s], sc.idx, sc.k)})
    return outs
