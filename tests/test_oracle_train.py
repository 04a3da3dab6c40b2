"""Pins of the oracle's training-step pieces (reconstruction loss with SSIM,
SGLD update, Philox4x32-10 noise) against published vectors, library
routines, closed forms and the defining distributions."""
import json
import os

import numpy as np
import pytest
import scipy.signal
import scipy.stats
import torch

from oracle import train

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    """Philox4x32-10 reproduces the generator's published known-answer vectors."""
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        ctr = np.array([[int(x, 16) for x in c["ctr"]]], np.uint32)
        key = tuple(int(x, 16) for x in c["key"])
        got = train.philox4x32(ctr, key)[0]
        assert [int(v) for v in got] == [int(x, 16) for x in c["out"]]


def test_philox_rounds_matter():
    """Fewer rounds give different words (the round count is part of the definition)."""
    ctr = np.array([[1, 2, 3, 4]], np.uint32)
    assert not np.array_equal(train.philox4x32(ctr, (5, 6), rounds=7), train.philox4x32(ctr, (5, 6)))


def test_normals_are_standard_normal():
    """Box-Muller output of consecutive counters passes a KS test against N(0,1)
    and has the normal's first four moments."""
    z = train.normals(np.arange(1 << 15, dtype=np.uint64), tag=3, step=7, seed=0x1234_5678_9abc).ravel()
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(scipy.stats.skew(z)) < 5 * np.sqrt(6 / n)
    assert abs(scipy.stats.kurtosis(z)) < 5 * np.sqrt(24 / n)
    # pairs from one counter are uncorrelated
    w = train.normals(np.arange(1 << 15, dtype=np.uint64), tag=3, step=7, seed=1)
    assert abs(np.corrcoef(w[:, 0], w[:, 1])[0, 1]) < 5 / np.sqrt(w.shape[0])


def test_noise_streams_are_distinct():
    """Tag, step, seed and index each select a different stream."""
    a = train.normals(np.arange(64, dtype=np.uint64), 1, 2, 3)
    for b in (train.normals(np.arange(64, dtype=np.uint64), 0, 2, 3),
              train.normals(np.arange(64, dtype=np.uint64), 1, 3, 3),
              train.normals(np.arange(64, dtype=np.uint64), 1, 2, 4),
              train.normals(np.arange(1, 65, dtype=np.uint64), 1, 2, 3)):
        assert np.abs(a - b).min() > 0


def test_sgld_proposal_mean_and_covariance():
    """The update is a draw from N(theta + eps/2 grad log p, eps I) with
    log p = -L: over many steps its sample mean and variance match."""
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(6)
    grad = rng.standard_normal(6)
    eps = 0.37
    steps = 4000
    draws = np.stack([train.sgld(theta, grad, eps, train.normals(np.arange(2, dtype=np.uint64), 9, s, 42).ravel()[:6])
                      for s in range(steps)])
    mean_expected = theta - 0.5 * eps * grad
    assert np.all(np.abs(draws.mean(0) - mean_expected) < 5 * np.sqrt(eps / steps))
    assert np.all(np.abs(draws.var(0) - eps) < 5 * eps * np.sqrt(2 / steps))


def test_sgld_zero_step_is_identity():
    theta = np.arange(5.0)
    assert np.array_equal(train.sgld(theta, np.ones(5), 0.0, np.ones(5)), theta)


def test_row_eps_columns():
    e = train.row_eps(0, 56, 1.0, 2.0, 3.0)
    assert np.all(e[:7] == 1.0) and e[7] == 2.0 and np.all(e[8:] == 3.0)
    assert np.all(train.row_eps(8, 48, 1.0, 2.0, 3.0) == 3.0)


def test_codebook_noise_layout():
    """Column c of row k uses normal c mod 4 of counter 16 k + c // 4."""
    z = train.codebook_noise(5, 0, 56, scene=2, step=3, seed=11)
    for k in (0, 4):
        for c in (0, 7, 8, 55):
            ref = train.normals(np.array([16 * k + c // 4], np.uint64), 0x10000 * 2 + 1, 3, 11)[0, c % 4]
            assert z[k, c] == ref
    z8 = train.codebook_noise(5, 8, 48, scene=2, step=3, seed=11)
    assert np.array_equal(z8, z[:, 8:])


# -------------------------------------------------------------------- SSIM
def test_ssim_window():
    g = train.ssim_window()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15 and np.allclose(g, g[::-1])
    assert np.argmax(g) == 5


def test_ssim_identical_images():
    """SSIM(x, x) = 1 everywhere, so the SSIM term and its gradient vanish."""
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (17, 23, 3))
    s = train.ssim_map(torch.tensor(x).permute(2, 0, 1), torch.tensor(x).permute(2, 0, 1))
    assert torch.allclose(s, torch.ones_like(s), atol=1e-12)
    loss, (g,) = train.loss_recon([x], [x], 1.0)
    assert abs(loss) < 1e-12 and np.abs(g).max() < 1e-12


def test_ssim_matches_scipy_convolution():
    """The same statistics from scipy.signal.convolve2d ('same', zero fill)."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (20, 31))
    y = np.clip(x + 0.1 * rng.standard_normal(x.shape), 0, 1)
    g = train.ssim_window()
    w = np.outer(g, g)
    cv = lambda a: scipy.signal.convolve2d(a, w, mode="same", boundary="fill", fillvalue=0.0)
    mx, my = cv(x), cv(y)
    sxx, syy, sxy = cv(x * x) - mx ** 2, cv(y * y) - my ** 2, cv(x * y) - mx * my
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    ref = (2 * mx * my + c1) * (2 * sxy + c2) / ((mx ** 2 + my ** 2 + c1) * (sxx + syy + c2))
    got = train.ssim_map(torch.tensor(x)[None], torch.tensor(y)[None])[0].numpy()
    assert np.abs(got - ref).max() < 1e-12


def test_ssim_constant_images_closed_form():
    """Constant images a, b: away from the border every variance vanishes and
    SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    x = torch.full((1, 30, 30), a, dtype=torch.float64)
    y = torch.full((1, 30, 30), b, dtype=torch.float64)
    s = train.ssim_map(x, y)[0]
    want = (2 * a * b + train.SSIM_C1) / (a * a + b * b + train.SSIM_C1)
    assert torch.allclose(s[5:-5, 5:-5], torch.full_like(s[5:-5, 5:-5], want), atol=1e-9)


def test_loss_recon_l1_only():
    """lambda = 0 is the mean absolute error (torch.nn.functional.l1_loss)."""
    rng = np.random.default_rng(3)
    x, t = rng.uniform(0, 1, (9, 10, 3)), rng.uniform(0, 1, (9, 10, 3))
    loss, (g,) = train.loss_recon([x], [t], 0.0)
    assert abs(loss - float(torch.nn.functional.l1_loss(torch.tensor(x), torch.tensor(t)))) < 1e-14
    assert np.allclose(g, np.sign(x - t) / x.size)


def test_loss_recon_gradient_finite_differences():
    rng = np.random.default_rng(4)
    ims = [rng.uniform(0, 1, (12, 13, 3)), rng.uniform(0, 1, (7, 16, 3))]
    tgs = [np.clip(im + 0.2 * rng.standard_normal(im.shape), 0, 1) for im in ims]
    lam = 0.2
    _, grads = train.loss_recon(ims, tgs, lam)
    h = 1e-6
    for v, (i, j, c) in ((0, (0, 0, 0)), (0, (6, 7, 1)), (1, (3, 15, 2)), (1, (0, 8, 0))):
        p = [im.copy() for im in ims]
        m = [im.copy() for im in ims]
        p[v][i, j, c] += h
        m[v][i, j, c] -= h
        fd = (train.loss_recon(p, tgs, lam)[0] - train.loss_recon(m, tgs, lam)[0]) / (2 * h)
        assert abs(fd - grads[v][i, j, c]) < 1e-7 * max(1.0, abs(fd)) + 1e-9
