"""Parity of the Metropolis-Hastings split and merge moves with the oracle,
through the C-ABI: live row count and every Gaussian's row index bit for bit,
row values within FP32 rounding of the oracle's FP64 (copies bit for bit),
the BF16 copy equal to round-to-nearest-even of the FP32 rows.  Seeds are
chosen so that no proposal's acceptance test lies within the oracle's
ambiguity margin of its threshold (asserted)."""
import numpy as np
import pytest
import torch

from oracle import mh
from paper_2509_03775_amd import cgs, render, scenes as sc
from harness import say

pytestmark = pytest.mark.gpu

ROW_TOL = 2e-6        # |gpu - oracle| / (1 + |value|) of a split row (c + u, u from FP32 normals)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cgs.load()
    yield
    torch.cuda.synchronize()


def _setup(rng, K_max, K, D, N, ld=None, mirror=True, dup_scale=None):
    ld = ld or D
    C = np.zeros((K_max, ld), np.float32)
    if dup_scale is None:
        C[:K, :D] = rng.standard_normal((K, D)).astype(np.float32)
    else:     # clusters of near-duplicate rows
        base = rng.standard_normal((max(2, K // 6), D))
        C[:K, :D] = (base[rng.integers(0, base.shape[0], K)] + dup_scale * rng.standard_normal((K, D))).astype(np.float32)
    idx = rng.integers(0, K, N).astype(np.int32)
    rows = torch.from_numpy(C).cuda()
    # the renderer's BF16 copy starts as RNE of the FP32 rows; moves refresh what they write
    mir = torch.from_numpy(sc.f32_to_bf16_bits(C).view(np.int16)).cuda() if mirror else None
    return C, idx, rows, mir


def _check(name, cbm: render.CodebookMoves, o, D, mir):
    torch.cuda.synchronize()
    K = cbm.live_rows()
    say(f"  {name}: K {K} (oracle {o['K']}), ambiguous {len(o['ambiguous'])}")
    assert not o["ambiguous"]
    assert K == o["K"]
    assert np.array_equal(cbm.idx.cpu().numpy().astype(np.int64), o["idx"])
    got = cbm.rows.cpu().numpy()[:K, :D].astype(np.float64)
    want = o["C"][:K, :D]
    err = np.max(np.abs(got - want) / (1 + np.abs(want))) if K else 0.0
    say(f"    row error {err:.2e}")
    assert err <= ROW_TOL
    if mir is not None:
        bits = mir.cpu().numpy().view(np.uint16)[:K, :D]
        assert np.array_equal(bits, sc.f32_to_bf16_bits(cbm.rows.cpu().numpy()[:K, :D]))


@pytest.mark.parametrize("D,ld,lam,eps", [(7, 7, 0.5, (0.1, 0.09)), (48, 48, 0.0, (0.1, 0.1)),
                                          (56, 64, 0.2, (0.05, 0.049))])
def test_split(D, ld, lam, eps):
    rng = np.random.default_rng(400 + D)
    K_max, K, N, B = 1500, 300, 20000, 1024
    seed, step = 0xABCDEF0123 + D, 17
    say(f"[split] D={D} lambda={lam} eps={eps}")
    C, idx, rows, mir = _setup(rng, K_max, K, D, N, ld)
    cbm = render.CodebookMoves(rows, K, torch.from_numpy(idx).cuda(), D=D, mirror=mir, n_proposals=B)
    cbm.split(cbm.params(lam, eps[0], eps[1], seed, step))
    o = mh.split(C[:, :D].astype(np.float64), K, idx, lam, eps[0], eps[1], B, step, seed)
    assert len(o["accepted"]) > 0
    _check("split", cbm, o, D, mir)


def test_split_capacity():
    rng = np.random.default_rng(9)
    K_max, K, D, N, B = 320, 300, 7, 5000, 512
    C, idx, rows, mir = _setup(rng, K_max, K, D, N)
    say("[split at capacity]")
    cbm = render.CodebookMoves(rows, K, torch.from_numpy(idx).cuda(), mirror=mir, n_proposals=B)
    cbm.split(cbm.params(0.0, 0.1, 0.1, 5, 6))
    o = mh.split(C.astype(np.float64), K, idx, 0.0, 0.1, 0.1, B, 6, 5)
    assert o["K"] == K_max
    _check("split", cbm, o, D, mir)


@pytest.mark.parametrize("D,dup", [(7, 0.01), (48, 0.004)])
def test_merge(D, dup):
    rng = np.random.default_rng(500 + D)
    K_max, K, N, B = 600, 480, 30000, 2048
    seed, step = 31337 + D, 3
    say(f"[merge] D={D}")
    C, idx, rows, mir = _setup(rng, K_max, K, D, N, dup_scale=dup)
    cbm = render.CodebookMoves(rows, K, torch.from_numpy(idx).cuda(), mirror=mir, n_proposals=B)
    cbm.merge(cbm.params(2.3, 0.1, 0.05, seed, step))
    o = mh.merge(C.astype(np.float64), K, idx, 2.3, 0.1, 0.05, B, step, seed)
    say(f"  merges {len(o['merges'])}")
    assert len(o["merges"]) > 10
    _check("merge", cbm, o, D, mir)
    # merged and moved rows are copies: bit for bit
    assert np.array_equal(cbm.rows.cpu().numpy()[:o["K"]], o["C"][:o["K"]].astype(np.float32))


def test_merge_degenerate_rows():
    """K = 1: nothing to merge; K = 2 identical rows: a merge whenever proposed."""
    for K in (1, 2):
        rng = np.random.default_rng(K)
        C = np.zeros((4, 3), np.float32)
        C[:K] = 0.25
        idx = rng.integers(0, K, 100).astype(np.int32)
        cbm = render.CodebookMoves(torch.from_numpy(C).cuda(), K, torch.from_numpy(idx).cuda(), n_proposals=8)
        cbm.merge(cbm.params(2.3, 0.1, 0.05, 1, 1))
        o = mh.merge(C.astype(np.float64), K, idx, 2.3, 0.1, 0.05, 8, 1, 1)
        _check(f"merge K={K}", cbm, o, 3, None)
        assert cbm.live_rows() == 1


def test_alternating_moves_keep_state_on_device():
    """Twelve moves (split and merge by the transition mixture's draw when it
    is not an update, else alternating), the live row count never leaving the
    device, against the oracle's sequence."""
    rng = np.random.default_rng(77)
    K_max, K, D, N, B = 2000, 500, 7, 40000, 512
    C, idx, rows, mir = _setup(rng, K_max, K, D, N, dup_scale=0.01)
    cbm = render.CodebookMoves(rows, K, torch.from_numpy(idx).cuda(), mirror=mir, n_proposals=B)
    Co, Ko, io = C.astype(np.float64), K, idx.astype(np.int64)
    seed = 2024
    say("[alternating moves]")
    for step in range(12):
        kind = {1: "split", 2: "merge"}.get(cgs.mh_transition(seed, step), "split" if step % 2 == 0 else "merge")
        p = cbm.params(0.3, 0.1, 0.08, seed, step)
        if kind == "split":
            cbm.split(p)
            o = mh.split(Co, Ko, io, 0.3, 0.1, 0.08, B, step, seed)
        else:
            cbm.merge(p)
            o = mh.merge(Co, Ko, io, 0.3, 0.1, 0.08, B, step, seed)
        assert not o["ambiguous"]
        Co, Ko, io = o["C"], o["K"], o["idx"]
    _check("after 12 moves", cbm, o, D, mir)
