"""Pins of the oracle's Metropolis-Hastings split and merge moves against the
transition mixture's probabilities, closed forms of the acceptance integrals
and the invariants of the moves."""
import math

import numpy as np
import pytest

from oracle import mh


def test_transition_mixture_frequencies():
    """Update / split / merge with probabilities 0.98 / 0.01 / 0.01."""
    n = 60000
    kinds = [mh.transition(12345, s) for s in range(n)]
    for name, p in (("update", 0.98), ("split", 0.01), ("merge", 0.01)):
        c = kinds.count(name)
        assert abs(c - n * p) < 5 * math.sqrt(n * p * (1 - p)), (name, c)


def test_choice_range():
    assert mh.choice(0, 7) == 0 and mh.choice(0xFFFFFFFF, 7) == 6
    w = np.random.default_rng(0).integers(0, 2 ** 32, 70000, dtype=np.uint64)
    c = np.array([mh.choice(int(x), 7) for x in w])
    counts = np.bincount(c, minlength=7)
    assert np.all(np.abs(counts - 10000) < 5 * math.sqrt(10000))


def _codebook(rng, K_max, K, D, N):
    C = np.zeros((K_max, D))
    C[:K] = rng.standard_normal((K, D))
    idx = rng.integers(0, K, N)
    return C, idx


def test_split_always_accepted_when_the_ratio_is_one():
    """lambda = 0 and eps_split = eps_merge make the acceptance 1: every
    distinct proposed Gaussian moves to a new row c + u, nothing else changes."""
    rng = np.random.default_rng(1)
    C, idx = _codebook(rng, 400, 100, 5, 3000)
    out = mh.split(C, 100, idx, lam=0.0, eps_split=0.1, eps_merge=0.1, B=250, step=3, seed=9)
    gs = [mh.choice(mh._words(16 * b, mh.SPLIT_TAG, 3, 9)[0], 3000) for b in range(250)]
    first = {}
    for b, g in enumerate(gs):
        first.setdefault(g, b)
    assert out["accepted"] == sorted(first.values())
    assert out["K"] == 100 + len(first)
    moved = set(first)
    for g in range(3000):
        if g in moved:
            b = first[g]
            assert out["idx"][g] >= 100
            assert np.allclose(out["C"][out["idx"][g]], C[idx[g]] + mh.split_offset(b, 5, 0.1, 3, 9), atol=0)
        else:
            assert out["idx"][g] == idx[g]
    assert np.array_equal(out["C"][:100], C[:100])


def test_split_capacity():
    rng = np.random.default_rng(2)
    C, idx = _codebook(rng, 110, 100, 3, 5000)
    out = mh.split(C, 100, idx, lam=0.0, eps_split=0.1, eps_merge=0.1, B=50, step=1, seed=4)
    assert out["K"] == 110 and len(out["accepted"]) == 10


def test_split_never_accepted_for_a_large_prior_cost():
    rng = np.random.default_rng(3)
    C, idx = _codebook(rng, 200, 100, 4, 1000)
    out = mh.split(C, 100, idx, lam=60.0, eps_split=0.1, eps_merge=0.05, B=500, step=2, seed=5)
    assert out["K"] == 100 and np.array_equal(out["idx"], idx)


def test_split_acceptance_rate_closed_form():
    """D = 1, lambda = 0: A = min(1, exp(-a u^2)), a = (1/eps_m^2 - 1/eps_s^2)/2,
    u ~ N(0, eps_s^2); E[A] = 1/sqrt(1 + 2 a eps_s^2) (Gaussian integral)."""
    eps_s, eps_m = 0.1, 0.05
    a = 0.5 * (1 / eps_m ** 2 - 1 / eps_s ** 2)
    want = 1.0 / math.sqrt(1.0 + 2.0 * a * eps_s ** 2)
    B = 20000
    acc = 0
    for b in range(B):
        w = mh._words(16 * b, mh.SPLIT_TAG, 7, 11)
        u = mh.split_offset(b, 1, eps_s, 7, 11)
        log_a = min(0.0, -mh.log_q_sm(float(u @ u), eps_s, eps_m))
        acc += math.log(float(mh.uniform24(w[1]))) < log_a
    assert abs(acc / B - want) < 5 * math.sqrt(want * (1 - want) / B)


def test_merge_selection_rate_closed_form():
    """Two rows at distance d: a single proposal always names the pair and
    merges it with probability exp(-d^2 / (2 eps_m^2)) (acceptance 1)."""
    d = 0.06
    C = np.zeros((2, 3))
    C[1, 0] = d
    want = math.exp(-d * d / (2 * 0.05 ** 2))
    steps = 6000
    hits = sum(len(mh.merge(C, 2, np.array([0, 1]), 2.3, 0.1, 0.05, 1, s, 21)["merges"]) for s in range(steps))
    assert abs(hits / steps - want) < 5 * math.sqrt(want * (1 - want) / steps)


def test_merge_invariants():
    """Identical rows merge whenever proposed; every row joins at most one
    merge; Gaussians keep their values or take their merge partner's; the live
    rows are compacted to 0 .. K'-1."""
    rng = np.random.default_rng(5)
    K, D, N = 64, 4, 2000
    base = rng.standard_normal((8, D))
    C = np.zeros((80, D))
    C[:K] = base[rng.integers(0, 8, K)]          # many exact duplicates
    idx = rng.integers(0, K, N)
    out = mh.merge(C, K, idx, lam=2.3, eps_split=0.1, eps_merge=0.05, B=40, step=8, seed=13)
    rows = [r for m in out["merges"] for r in m]
    assert len(rows) == len(set(rows)) and len(out["merges"]) > 0
    assert out["K"] == K - len(out["merges"])
    assert out["idx"].min() >= 0 and out["idx"].max() < out["K"]
    partner = {c2: c for c, c2 in out["merges"]}
    for g in range(N):
        old = idx[g]
        want = C[partner.get(old, old)]
        assert np.array_equal(out["C"][out["idx"][g]], want)
    live = {tuple(C[r]) for r in range(K) if r not in partner}
    assert {tuple(out["C"][r]) for r in range(out["K"])} <= live


def test_merge_far_rows_never_merge():
    rng = np.random.default_rng(6)
    C, idx = _codebook(rng, 50, 50, 6, 500)
    out = mh.merge(C * 10, 50, idx, 2.3, 0.1, 0.05, 200, 1, 3)
    assert out["merges"] == [] and out["K"] == 50 and np.array_equal(out["idx"], idx)
