"""ORACLE (test infrastructure only): the training-step pieces around the
render -- the reconstruction loss with its SSIM term and the SGLD parameter
update with its Gaussian noise.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does.  It shares no code with the HIP
path.

* Reconstruction loss (paper Sec. 2.1, Eq. 4):
      L = (1 - lambda) L1 + lambda L_SSIM,   L_SSIM = 1 - mean SSIM,
  the means taken over every pixel and colour channel.  SSIM is the
  structural similarity of Wang et al. (2004) with its usual constants: an
  11x11 Gaussian window of standard deviation 1.5 (normalised), C1 = 0.01^2,
  C2 = 0.03^2 for a dynamic range of 1, local statistics by "same"-size
  convolution with zero padding, per channel.  The gradient is PyTorch
  autograd of this definition in FP64.
* SGLD parameter update (paper Sec. 2.3 and the parameter-update transition
  of Sec. 4.4 / App. A.1):
      theta' = theta + (eps / 2) grad log p + sqrt(eps) eta,  eta ~ N(0, I),
  with log p = -L + const, i.e. theta' = theta - (eps/2) dL/dtheta + sqrt(eps) eta,
  one step size per parameter kind (means, opacity, SR codebook, SH codebook).
* The noise eta is drawn from the counter-based generator Philox4x32-10
  (Salmon, Moraes, Dror and Shaw, SC 2011) and turned into normals by the
  Box-Muller transform, so that any implementation of the same published
  definitions reproduces it: counter (index lo, index hi, tag, step), key =
  the 64-bit seed (lo, hi); output words (w0, w1) give (z0, z1) and (w2, w3)
  give (z2, z3) with u = ((w >> 9) + 1/2) 2^-23, r = sqrt(-2 ln u_a),
  z = r cos(2 pi u_b), r sin(2 pi u_b).
  Per Gaussian g of scene s: index g, tag 0x10000 s; z0..z2 -> the mean's
  x, y, z and z3 -> the per-Gaussian opacity logit.  Codebook row k of
  scene s, row-layout column c (ls 0-2, q 3-6, logit 7, SH 8-): index
  16 k + c // 4, tag 0x10000 s + 1, normal z_{c mod 4}.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np
import torch

# ------------------------------------------------------------ Philox4x32-10
_M0, _M1 = 0xD2511F53, 0xCD9E8D57          # round multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85          # key (Weyl) increments
_MASK = 0xFFFFFFFF


def philox4x32(ctr: np.ndarray, key: Tuple[int, int], rounds: int = 10) -> np.ndarray:
    """Philox4x32 of counters ctr uint32[n, 4] under key (k0, k1): uint32[n, 4].
    Each round multiplies words 0 and 2 by the round multipliers, keeps the
    low halves as new words 1 and 3 and xors the high halves with the other
    two words and the key into new words 0 and 2; the key is bumped by the
    Weyl increments between rounds."""
    x = [ctr[:, i].astype(np.uint64) for i in range(4)]
    k0 = np.uint64(key[0] & _MASK)
    k1 = np.uint64(key[1] & _MASK)
    m0, m1 = np.uint64(_M0), np.uint64(_M1)
    mask = np.uint64(_MASK)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + np.uint64(_W0)) & mask
            k1 = (k1 + np.uint64(_W1)) & mask
        p0 = m0 * x[0]
        p1 = m1 * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        x = [(hi1 ^ x[1] ^ k0) & mask, lo1, (hi0 ^ x[3] ^ k1) & mask, lo0]
    return np.stack(x, 1).astype(np.uint32)


def box_muller(w: np.ndarray) -> np.ndarray:
    """uint32[n, 4] -> float64[n, 4] standard normals (pairs (w0,w1), (w2,w3))."""
    u = ((w >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    out = np.empty(w.shape, np.float64)
    for a, b in ((0, 1), (2, 3)):
        r = np.sqrt(-2.0 * np.log(u[:, a]))
        t = 2.0 * math.pi * u[:, b]
        out[:, a] = r * np.cos(t)
        out[:, b] = r * np.sin(t)
    return out


def normals(index: np.ndarray, tag: int, step: int, seed: int) -> np.ndarray:
    """The four normals of each counter (index, tag, step): float64[n, 4]."""
    index = np.asarray(index, np.uint64)
    ctr = np.stack([(index & np.uint64(_MASK)).astype(np.uint32),
                    (index >> np.uint64(32)).astype(np.uint32),
                    np.full(index.shape, tag & _MASK, np.uint32),
                    np.full(index.shape, step & _MASK, np.uint32)], 1)
    return box_muller(philox4x32(ctr, (seed & _MASK, (seed >> 32) & _MASK)))


def gaussian_noise(n: int, scene: int, step: int, seed: int) -> np.ndarray:
    """Per-Gaussian noise float64[n, 4]: columns mean x, y, z, opacity logit."""
    return normals(np.arange(n, dtype=np.uint64), 0x10000 * scene, step, seed)


def codebook_noise(rows: int, col0: int, ncols: int, scene: int, step: int, seed: int) -> np.ndarray:
    """Noise float64[rows, ncols] of row-layout columns col0 .. col0+ncols-1."""
    out = np.empty((rows, ncols), np.float64)
    k = np.arange(rows, dtype=np.uint64)
    for j in range(ncols):
        c = col0 + j
        z = normals(16 * k + np.uint64(c // 4), 0x10000 * scene + 1, step, seed)
        out[:, j] = z[:, c % 4]
    return out


def sgld(theta: np.ndarray, grad: np.ndarray, eps, noise: np.ndarray) -> np.ndarray:
    """One SGLD step theta - (eps/2) dL/dtheta + sqrt(eps) eta (log p = -L);
    eps broadcasts against theta (one step size per column allowed)."""
    eps = np.asarray(eps, np.float64)
    return np.asarray(theta, np.float64) - 0.5 * eps * np.asarray(grad, np.float64) + np.sqrt(eps) * noise


def row_eps(col0: int, ncols: int, eps_sr: float, eps_opacity: float, eps_sh: float) -> np.ndarray:
    """Step size of each row-layout column: ls and q -> SR, logit -> opacity,
    SH -> SH."""
    c = np.arange(col0, col0 + ncols)
    return np.where(c < 7, eps_sr, np.where(c == 7, eps_opacity, eps_sh)).astype(np.float64)


# -------------------------------------------------------------------- SSIM
SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window() -> np.ndarray:
    """The normalised 1-D Gaussian of the separable 11x11 window."""
    x = np.arange(SSIM_WINDOW, dtype=np.float64) - SSIM_WINDOW // 2
    g = np.exp(-x * x / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _blur(x: torch.Tensor) -> torch.Tensor:
    """'same' convolution of [C, H, W] with the 11x11 window, zero padding."""
    g = torch.from_numpy(ssim_window())
    w2 = torch.outer(g, g)[None, None].to(x.dtype)
    c = x.shape[0]
    return torch.nn.functional.conv2d(x[:, None], w2, padding=SSIM_WINDOW // 2).reshape(c, *x.shape[1:])


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Per-pixel, per-channel SSIM of images [C, H, W]."""
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def loss_recon(images, targets, lam: float):
    """Eq. 4 over a batch of views: images/targets lists of float[H, W, 3].
    Returns (loss, [dL/dimage float64[H, W, 3]]).  L1 and SSIM are each the
    mean over all pixels and channels of the batch (sign(0) = 0 for L1)."""
    xs = [torch.tensor(np.asarray(im, np.float64), requires_grad=True) for im in images]
    n = sum(x.numel() for x in xs)
    l1 = sum((x - torch.tensor(np.asarray(t, np.float64))).abs().sum() for x, t in zip(xs, targets)) / n
    s = sum(ssim_map(x.permute(2, 0, 1), torch.tensor(np.asarray(t, np.float64)).permute(2, 0, 1)).sum()
            for x, t in zip(xs, targets)) / n
    loss = (1.0 - lam) * l1 + lam * (1.0 - s)
    loss.backward()
    return float(loss.detach()), [x.grad.numpy() for x in xs]
