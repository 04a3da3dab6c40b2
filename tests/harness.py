"""Shared helpers of the parity tests: run the HIP path through its Python
binding, run the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import sys
from typing import Dict, List, Optional, Sequence

import numpy as np

import oracle
from paper_2509_03775_amd import scenes as sc

IMAGE_TOL = 1e-4          # max |gpu - oracle| on non-ambiguous pixels
GRAD_TOL = 1e-3           # relative L2 error per parameter block

BLOCKS = {"ls": slice(0, 3), "q": slice(3, 7), "logit": slice(7, 8), "sh_dc": slice(8, 11), "sh_rest": slice(11, None)}


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def grad_errors(gpu_means, gpu_cb, ora_means, ora_cb) -> Dict[str, float]:
    out = {"means": rel_l2(gpu_means, ora_means)}
    for k, s in BLOCKS.items():
        if ora_cb[:, s].size:
            out[k] = rel_l2(gpu_cb[:, s], ora_cb[:, s])
    return out


def grad_error_stats(gpu_means, gpu_cb, ora_means, ora_cb) -> Dict[str, Dict[str, float]]:
    """Per parameter block: relative L2 error, and the 99th percentile and
    maximum of the element-wise relative error |g - o| / (|o| + 1e-6 max|o|)."""
    out = {}
    pairs = [("means", gpu_means, ora_means)] + [(k, gpu_cb[:, s], ora_cb[:, s]) for k, s in BLOCKS.items()]
    for k, g, o in pairs:
        g = np.asarray(g, np.float64).ravel()
        o = np.asarray(o, np.float64).ravel()
        if not o.size:
            continue
        e = np.abs(g - o) / (np.abs(o) + 1e-6 * max(np.abs(o).max(), 1e-300))
        out[k] = {"rel_l2": rel_l2(g, o), "p99": float(np.percentile(e, 99)), "max": float(e.max())}
    return out


def record(kind: str, **fields) -> None:
    """One machine-readable line of measured parity errors (collected into the
    design notes' error table)."""
    import json
    say("PARITY " + json.dumps({"case": kind, **fields}, sort_keys=True))


def random_tiles(cam, n_tiles: int, seed: int) -> np.ndarray:
    """Pixels of n_tiles random 16x16 tiles of a view (clipped to the image)."""
    rng = np.random.default_rng(seed)
    tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
    pick = rng.choice(tx * ty, size=min(n_tiles, tx * ty), replace=False)
    pix = []
    for t in pick:
        x0, y0 = (t % tx) * 16, (t // tx) * 16
        yy, xx = np.mgrid[y0:min(y0 + 16, cam.height), x0:min(x0 + 16, cam.width)]
        pix.append(np.stack([xx.ravel(), yy.ravel()], 1))
    return np.concatenate(pix).astype(np.int32)


def full_pixels(cam) -> np.ndarray:
    yy, xx = np.mgrid[0:cam.height, 0:cam.width]
    return np.stack([xx.ravel(), yy.ravel()], 1).astype(np.int32)


def oracle_grad_image(wl: sc.Workload, pix: Sequence[np.ndarray], outs: List[dict]):
    """dL/dC of the L1 loss at the sampled pixels (normalised by the full
    image size), zero at ambiguous pixels; returns per-view [n_pix,3] arrays
    and the full [P,3] image-gradient array for the GPU."""
    P = wl.n_pixels
    per_view, full = [], np.zeros((P, 3), np.float32)
    off = 0
    for v, cam in enumerate(wl.cameras):
        o = outs[v]
        tgt = wl.targets[v][pix[v][:, 1], pix[v][:, 0]].astype(np.float64)
        g = np.sign(o["color"] - tgt) / (3.0 * P)
        g[o["ambiguous"]] = 0.0
        g32 = g.astype(np.float32)
        per_view.append(g32.astype(np.float64))
        lin = off + pix[v][:, 1].astype(np.int64) * cam.width + pix[v][:, 0]
        full[lin] = g32
        off += cam.width * cam.height
    return per_view, full


def oracle_render(wl: sc.Workload, pix: Sequence[np.ndarray], grad_colors=None) -> List[dict]:
    outs = []
    for v, cam in enumerate(wl.cameras):
        s = wl.scenes[int(wl.view_scene[v])]
        gcol = None if grad_colors is None else grad_colors[v]
        outs.append(oracle.render_view(s, cam, pix[v], grad_color=gcol))
    return outs


def oracle_scene_grads(wl: sc.Workload, outs: List[dict]):
    gm = [np.zeros((s.n, 3)) for s in wl.scenes]
    gr = [np.zeros((s.n, s.r)) for s in wl.scenes]
    for v, o in enumerate(outs):
        s = int(wl.view_scene[v])
        gm[s] += o["grad_means"]
        gr[s] += o["grad_rows"]
    gcb = [oracle.codebook_grad_reduce(gr[i], s.idx, s.k) for i, s in enumerate(wl.scenes)]
    return gm, gcb


def compare_view(gpu_img: np.ndarray, gpu_T: np.ndarray, gpu_nl: np.ndarray, cam, pix: np.ndarray, o: dict):
    """Returns (max abs colour error on non-ambiguous pixels, T error,
    #n_last mismatches on non-ambiguous pixels, #ambiguous)."""
    g = gpu_img.reshape(cam.height, cam.width, 3)[pix[:, 1], pix[:, 0]].astype(np.float64)
    t = gpu_T.reshape(cam.height, cam.width)[pix[:, 1], pix[:, 0]].astype(np.float64)
    nl = gpu_nl.reshape(cam.height, cam.width)[pix[:, 1], pix[:, 0]]
    ok = ~o["ambiguous"]
    ec = float(np.abs(g[ok] - o["color"][ok]).max()) if ok.any() else 0.0
    et = float(np.abs(t[ok] - o["T"][ok]).max()) if ok.any() else 0.0
    mism = int((nl[ok] != o["n_last"][ok]).sum())
    return ec, et, mism, int((~ok).sum())
