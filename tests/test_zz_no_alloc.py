"""The allocation-free codebook reduction (cgs_codebook_grad_reduce_noalloc)
against the workspace entry point (cgs_codebook_grad_reduce), through the
C-ABI: the same kernels, so the same bits, on two calls in a row -- the
second smaller, so it runs on what the first left in the library's device
scratch -- plus the oracle's FP64 sums, and the host-side refusal of sizes
beyond the fixed scratch."""
import zlib

import numpy as np
import pytest
import torch

import oracle
from paper_2509_03775_amd import cgs
from harness import say

pytestmark = pytest.mark.gpu


def _dev(a, dt=None):
    return torch.from_numpy(np.ascontiguousarray(a if dt is None else a.astype(dt))).cuda()


def _both(g, idx, k, perm=None):
    n, d = g.shape
    dg, di = _dev(g, np.float32), _dev(idx, np.int32)
    dp = _dev(perm, np.int32) if perm is not None else None
    st = torch.cuda.current_stream().cuda_stream
    want = torch.full((k, d), 7.0, dtype=torch.float32, device="cuda")
    nb = cgs.codebook_grad_reduce_workspace_bytes(n, k, d)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    cgs.codebook_grad_reduce(dg.data_ptr(), d, di.data_ptr(), cgs.ptr(dp), n, k, d, want.data_ptr(), d,
                             ws.data_ptr(), nb, st)
    got = torch.full((k, d), -3.0, dtype=torch.float32, device="cuda")
    cgs.codebook_grad_reduce_noalloc(dg.data_ptr(), d, di.data_ptr(), cgs.ptr(dp), n, k, d, got.data_ptr(), d, st)
    torch.cuda.synchronize()
    return got.cpu().numpy(), want.cpu().numpy()


@pytest.mark.parametrize("perm", [False, True])
def test_noalloc_reduce_matches_workspace_entry_point(perm):
    rng = np.random.default_rng(zlib.crc32(b"noalloc") + int(perm))
    # first call large (a Zipf-skewed index: long runs of one row), the second
    # smaller with other rows, so it reads scratch the first call filled
    for n, k, d in [(600000, 16384, 56), (70001, 777, 11)]:
        say(f"[noalloc reduce] n={n} k={k} d={d} perm={perm}")
        idx = np.minimum(rng.zipf(1.2, n) - 1, k - 1) if n > 100000 else rng.integers(0, k, n)
        g = rng.standard_normal((n, d)).astype(np.float32)
        p = np.argsort(idx, kind="stable") if perm else None
        got, want = _both(g, idx, k, p)
        np.testing.assert_array_equal(got, want)
        ref = oracle.codebook_grad_reduce(g.astype(np.float64), idx, k)
        scale = np.sqrt(np.bincount(idx, minlength=k).max() + 1.0)
        assert np.abs(got - ref).max() <= 4e-5 * scale


def test_noalloc_reduce_limits():
    say("[noalloc reduce] limits")
    L = cgs.load()
    # beyond the 32 MiB scratch: refused on the host before any launch
    n = 4_000_000
    assert cgs.codebook_grad_reduce_workspace_bytes(n, 65536, 56) > 32 << 20
    assert L.cgs_codebook_grad_reduce_noalloc(0x1, 56, 0x2, None, n, 65536, 56, 0x3, 56, None) == cgs.CGS_ELIMIT
    assert L.cgs_codebook_grad_reduce_noalloc(0x1, 56, 0x2, None, 10, 0, 56, 0x3, 56, None) == cgs.CGS_EINVAL
    # the largest size that fits, and an empty input, still run
    n = 1_800_000
    assert cgs.codebook_grad_reduce_workspace_bytes(n, 65536, 8) <= 32 << 20
    rng = np.random.default_rng(5)
    idx = rng.integers(0, 65536, n)
    g = rng.standard_normal((n, 8)).astype(np.float32)
    got, want = _both(g, idx, 65536)
    np.testing.assert_array_equal(got, want)
    got, want = _both(np.zeros((0, 8), np.float32), np.zeros(0, np.int64), 5)
    np.testing.assert_array_equal(got, np.zeros((5, 8), np.float32))
    np.testing.assert_array_equal(want, np.zeros((5, 8), np.float32))
