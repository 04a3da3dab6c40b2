"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module draws random numbers and lays them out; it holds none of the
renderer's arithmetic (no projection, no compositing, no activation).  The
scenes stand in for the multi-view datasets the paper trains on (Sec. 5.1),
which are not available here; their shapes follow the paper's scale
(millions of Gaussians, codebook-indexed parameters, Sec. 4.1).

Codebook row layout (one fused codebook, one int32 index per Gaussian):
    [log-scale 3, quaternion 4 (w,x,y,z), opacity logit 1, SH 3*(d+1)^2]
with SH stored coefficient-major, RGB-minor: sh[j*3 + ch], j = l*l + l + m.
The paper's state (Sec. 4.1, state S={G,C}) keeps the scale+quaternion part
and the SH part in two codebooks; the row above holds both halves.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


def row_width(sh_degree: int) -> int:
    return 8 + 3 * (sh_degree + 1) ** 2


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even float32 -> bfloat16 storage bits (uint16)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)
    return r


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    Rt: np.ndarray        # float32 [3,4] world->camera, row-major [R|t]
    campos: np.ndarray    # float32 [3]
    bg: np.ndarray        # float32 [3]

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    means: np.ndarray      # float32 [N,3]
    idx: np.ndarray        # int32 [N]
    cb: np.ndarray         # float32 [K,R] (values the renderer reads)
    sh_degree: int
    cb_bf16: Optional[np.ndarray] = None   # uint16 [K,R] storage bits when BF16

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def k(self) -> int:
        return int(self.cb.shape[0])

    @property
    def r(self) -> int:
        return int(self.cb.shape[1])


@dataclasses.dataclass
class Workload:
    name: str
    scenes: List[Scene]
    cameras: List[Camera]
    view_scene: np.ndarray    # int32 [V]: scene of each view
    targets: List[np.ndarray]  # float32 [H,W,3] per view
    bf16: bool

    @property
    def n_pixels(self) -> int:
        return sum(c.n_pixels for c in self.cameras)


def pinhole(width: int, height: int, eye, target=(0.0, 0.0, 0.0), up=(0.0, -1.0, 0.0)) -> Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward), 60 deg
    horizontal field of view, principal point at the image centre."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, dtype=np.float64)
    right = np.cross(fwd, upv)
    if np.linalg.norm(right) < 1e-9:
        right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd], axis=0)
    t = -R @ eye
    Rt = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
    f = (width / 2.0) / math.tan(math.radians(30.0))
    return Camera(width, height, np.float32(f), np.float32(f),
                  np.float32((width - 1) / 2.0), np.float32((height - 1) / 2.0),
                  Rt, eye.astype(np.float32), np.zeros(3, np.float32))


def _random_rotations(rng, n):
    """Random proper rotations from the QR factorisation of Gaussian matrices."""
    out = np.empty((n, 3, 3))
    for i in range(n):
        qm, rm = np.linalg.qr(rng.standard_normal((3, 3)))
        qm = qm * np.sign(np.diag(rm))[None, :]
        if np.linalg.det(qm) < 0:
            qm[:, 0] = -qm[:, 0]
        out[i] = qm
    return out


def clustered_means(rng, n, n_clusters=32):
    """Mixture of anisotropic Gaussian clusters: centres U[-1,1]^3, per-cluster
    axis sigmas U(0.03,0.25)^3 in a random frame, equal weights."""
    centres = rng.uniform(-1.0, 1.0, (n_clusters, 3))
    sig = rng.uniform(0.03, 0.25, (n_clusters, 3))
    frames = _random_rotations(rng, n_clusters)
    which = rng.integers(0, n_clusters, n)
    z = rng.standard_normal((n, 3)) * sig[which]
    return centres[which] + np.einsum("nij,nj->ni", frames[which], z)


def make_scene(rng, n, k, sh_degree, mu_s, clusters, bf16=False, sigma_s=0.5) -> Scene:
    if clusters:
        means = clustered_means(rng, n)
    else:
        means = rng.uniform(-1.0, 1.0, (n, 3))
    R = row_width(sh_degree)
    cb = np.zeros((k, R))
    cb[:, 0:3] = rng.normal(mu_s, sigma_s, (k, 3))
    q = rng.standard_normal((k, 4))
    cb[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    cb[:, 7] = rng.standard_normal(k)
    cb[:, 8:11] = rng.uniform(0.0, 1.0, (k, 3))
    if sh_degree > 0:
        cb[:, 11:] = rng.normal(0.0, 0.05, (k, R - 11))
    idx = rng.integers(0, k, n).astype(np.int32)
    cb32 = cb.astype(np.float32)
    bits = None
    if bf16:
        bits = f32_to_bf16_bits(cb32)
        cb32 = bf16_bits_to_f32(bits)
    return Scene(means.astype(np.float32), idx, np.ascontiguousarray(cb32), sh_degree, bits)


def screen_matched_mu(width: int) -> float:
    """Log-scale mean that keeps the median projected footprint of the
    128-px reference scene at every resolution."""
    return -3.0 + math.log(128.0 / width)


def _targets(rng, cams):
    return [rng.uniform(0.0, 1.0, (c.height, c.width, 3)).astype(np.float32) for c in cams]


WORKLOADS = ("uniform4k_128px", "clusters200k_800px", "clusters1m_1600x1064",
             "clusters4m_bf16_4x1957x1091", "uneven16_512px")


def make_workload(name: str, bf16: Optional[bool] = None, n_override: Optional[int] = None) -> Workload:
    """Build one of the named synthetic workloads (seeded, deterministic).

    bf16 overrides the codebook storage type (the 4M and 16-scene workloads
    default to BF16, the others to FP32); n_override shrinks N for quick runs.
    """
    seed = 1000 + WORKLOADS.index(name) + 1
    rng = np.random.default_rng(seed)
    if name == "uniform4k_128px":
        n, k, d, W, H = 4096, 256, 0, 128, 128
        sc = make_scene(rng, n_override or n, k, d, -3.0, clusters=False, bf16=bool(bf16))
        cams = [pinhole(W, H, (0.0, 0.0, -3.0))]
        vs = [0]
        scenes = [sc]
        use_bf16 = bool(bf16)
    elif name in ("clusters200k_800px", "clusters1m_1600x1064"):
        if name == "clusters200k_800px":
            n, k, W, H = 200_000, 4096, 800, 800
        else:
            n, k, W, H = 1_000_000, 16384, 1600, 1064
        use_bf16 = bool(bf16)
        sc = make_scene(rng, n_override or n, k, 3, screen_matched_mu(W), clusters=True, bf16=use_bf16)
        cams = [pinhole(W, H, (0.0, 0.0, -3.0))]
        vs = [0]
        scenes = [sc]
    elif name == "clusters4m_bf16_4x1957x1091":
        n, k, W, H = 4_000_000, 65536, 1957, 1091
        use_bf16 = True if bf16 is None else bool(bf16)
        sc = make_scene(rng, n_override or n, k, 3, screen_matched_mu(W), clusters=True, bf16=use_bf16)
        cams = []
        for az in (0.0, 90.0, 180.0, 270.0):
            a = math.radians(az)
            eye = (3.0 * math.sin(a), 0.0, -3.0 * math.cos(a))
            cams.append(pinhole(W, H, eye))
        vs = [0, 0, 0, 0]
        scenes = [sc]
    elif name == "uneven16_512px":
        use_bf16 = True if bf16 is None else bool(bf16)
        W = H = 512
        scenes, cams, vs = [], [], []
        for s in range(16):
            ns = int(round(math.exp(rng.uniform(math.log(50_000), math.log(500_000)))))
            ks = int(round(math.exp(rng.uniform(math.log(1024), math.log(8192)))))
            if n_override:
                ns = max(1, min(ns, n_override))
            scenes.append(make_scene(rng, ns, ks, 3, screen_matched_mu(W), clusters=True, bf16=use_bf16))
            cams.append(pinhole(W, H, (0.0, 0.0, -3.0)))
            vs.append(s)
    else:
        raise KeyError(name)
    return Workload(name, scenes, cams, np.asarray(vs, np.int32), _targets(rng, cams), use_bf16)


def random_scene(seed: int, n: int, k: int, sh_degree: int, mu_s: float = -3.0,
                 clusters: bool = False, bf16: bool = False) -> Scene:
    """Small seeded scene for unit tests."""
    return make_scene(np.random.default_rng(seed), n, k, sh_degree, mu_s, clusters, bf16)


def needle_scene(seed: int, n_needles: int = 12, n_background: int = 3000, k_background: int = 64,
                 sh_degree: int = 1, ratio: float = 2000.0) -> Scene:
    """Small seeded scene seen from (0,0,-3) with n_needles "needle" Gaussians:
    one long axis lying in a plane facing the camera at an on-screen angle
    drawn from 30-60 or 120-150 degrees, the two short axes `ratio` times
    shorter, each on a codebook row of its own, plus n_background ordinary
    Gaussians (uniform in [-1,1]^3) on k_background shared rows.  The needles'
    projected footprints are elongated enough that the 2x2 determinant of
    their projected covariance nearly cancels (the near-degenerate case)."""
    rng = np.random.default_rng(seed)
    R = row_width(sh_degree)
    bg = make_scene(rng, n_background, k_background, sh_degree, -3.5, clusters=False)
    cb = np.zeros((n_needles, R))
    long_ls = np.log(rng.uniform(0.45, 0.75, n_needles))
    cb[:, 0] = long_ls
    cb[:, 1] = long_ls - math.log(ratio)
    cb[:, 2] = long_ls - math.log(ratio)
    ang = np.where(rng.uniform(size=n_needles) < 0.5, rng.uniform(30.0, 60.0, n_needles),
                   rng.uniform(120.0, 150.0, n_needles))
    half = np.radians(ang) / 2.0
    cb[:, 3] = np.cos(half)          # rotation about the viewing axis (w, 0, 0, sin)
    cb[:, 6] = np.sin(half)
    cb[:, 7] = rng.normal(1.0, 0.5, n_needles)
    cb[:, 8:11] = rng.uniform(0.0, 1.0, (n_needles, 3))
    if sh_degree > 0:
        cb[:, 11:] = rng.normal(0.0, 0.05, (n_needles, R - 11))
    nm = np.stack([rng.uniform(-0.6, 0.6, n_needles), rng.uniform(-0.4, 0.4, n_needles),
                   rng.uniform(-0.5, 0.5, n_needles)], 1)
    means = np.concatenate([bg.means.astype(np.float64), nm]).astype(np.float32)
    idx = np.concatenate([bg.idx, k_background + np.arange(n_needles, dtype=np.int32)]).astype(np.int32)
    cb_all = np.concatenate([bg.cb.astype(np.float64), cb]).astype(np.float32)
    return Scene(means, idx, np.ascontiguousarray(cb_all), sh_degree, None)
