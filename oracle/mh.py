"""ORACLE (test infrastructure only): the Metropolis-Hastings split and merge
moves on a codebook (paper Sec. 4.4 and App. A.1), as plain sequential loops
in FP64.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does.  It shares no code with the HIP
path.

What a move does (readings of the paper's text, which gives the proposal and
acceptance of one split or one merge but not how many are made per step):

* Transition mixture: each training step is a parameter update with
  probability 0.98, a split step with 0.01 and a merge step with 0.01, drawn
  from u = uniform24(word 0) of the Philox counter (0, 0, 0x20002, step).
* A split or merge step makes B independent proposals; proposal b reads the
  Philox counters 16 b + j (j = 0..15), tag 0x20000 (split) / 0x20001
  (merge), the step, the seed.  Counter j = 0 gives the choices and the
  acceptance uniform, counters j = 1..15 the normals of the split offset u
  (u_d = eps_split z_{d}, z taken in order, four per counter).
* Integer choices by multiply-shift: floor(w n / 2^32) for a word w, exact.
  uniform24(w) = ((w >> 8) + 1/2) 2^-24.
* Split proposal: Gaussian g = choice(w0, N); offset u ~ N(0, eps_split^2 I)
  over the row's D values; acceptance (paper): A = min(1, e^-lambda / q_sm(u))
  with q_sm(u) = exp(-|u|^2/2 (1/eps_split^2 - 1/eps_merge^2)); accepted iff
  log uniform24(w1) < log A.  Among accepted proposals a Gaussian splits once
  (the lowest b naming it); the survivors in b order get new rows K, K+1, ...
  while rows remain (K < K_max): new row = C[idx[g]] + u, idx[g] = new row.
  The original row keeps its value (c' = c, c'' = c + u).
* Merge proposal: rows c = choice(w0, K), c' = choice(w1, K - 1), c' += 1 if
  c' >= c (a uniform ordered pair of distinct rows).  The pair is selected
  with the thinning probability exp(-|c - c'|^2 / (2 eps_merge^2)), which makes
  selected pairs distributed as q_merge = N(c - c'; 0, eps_merge^2 I), and
  accepted with A = min(1, e^lambda q_sm(c - c')); both as one test:
  log uniform24(w2) < -|c - c'|^2 / (2 eps_merge^2) + log A.  A row takes part
  in at most one merge per step: a proposal is withdrawn if an earlier
  accepted proposal (lower b) names either of its rows.  Each surviving merge
  remaps the Gaussians of c' to c (c keeps its value) and frees c'.
* Compaction after merges: with K' = K - (number of merges), the freed rows
  below K' (ascending) receive the surviving rows at or above K' (ascending)
  -- row values and the Gaussians mapped to them move together -- so the live
  rows stay 0 .. K'-1.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

from .train import box_muller, philox4x32

SPLIT_TAG, MERGE_TAG, MIX_TAG = 0x20000, 0x20001, 0x20002
P_UPDATE, P_SPLIT = 0.98, 0.01


def uniform24(w) -> np.ndarray:
    return ((np.asarray(w, np.uint32) >> np.uint32(8)).astype(np.float64) + 0.5) * 2.0 ** -24


def choice(w, n: int) -> int:
    """floor(w n / 2^32): an integer uniform over [0, n)."""
    return int((int(w) * int(n)) >> 32)


def _words(index: int, tag: int, step: int, seed: int) -> np.ndarray:
    ctr = np.array([[index & 0xFFFFFFFF, (index >> 32) & 0xFFFFFFFF, tag, step & 0xFFFFFFFF]], np.uint32)
    return philox4x32(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))[0]


def transition(seed: int, step: int) -> str:
    """'update', 'split' or 'merge' for a training step (0.98 / 0.01 / 0.01)."""
    u = float(uniform24(_words(0, MIX_TAG, step, seed)[0]))
    return "update" if u < P_UPDATE else ("split" if u < P_UPDATE + P_SPLIT else "merge")


def split_offset(b: int, D: int, eps_split: float, step: int, seed: int) -> np.ndarray:
    ctr = np.array([[16 * b + j, 0, SPLIT_TAG, step] for j in range(1, 16)], np.uint32)
    z = box_muller(philox4x32(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))).ravel()
    return eps_split * z[:D]


def log_q_sm(u2: float, eps_split: float, eps_merge: float) -> float:
    """log q_sm of an offset with squared norm u2."""
    return -0.5 * u2 * (1.0 / eps_split ** 2 - 1.0 / eps_merge ** 2)


def split(C: np.ndarray, K: int, idx: np.ndarray, lam: float, eps_split: float, eps_merge: float, B: int,
          step: int, seed: int, margin: float = 1e-5) -> Dict:
    """One batched split step.  C float64 [K_max, D] (rows >= K unused), idx
    int [N].  Returns the new C, K, idx, the accepted proposals and the
    proposals whose acceptance test was within `margin` (relative) of its
    threshold (where FP32 may decide differently)."""
    C = np.array(C, np.float64)
    idx = np.array(idx, np.int64)
    K_max, D = C.shape
    N = idx.shape[0]
    accepted, ambiguous, taken = [], [], set()
    for b in range(B):
        w = _words(16 * b, SPLIT_TAG, step, seed)
        g = choice(w[0], N)
        u = split_offset(b, D, eps_split, step, seed)
        log_a = min(0.0, -lam - log_q_sm(float(u @ u), eps_split, eps_merge))
        lu = math.log(float(uniform24(w[1])))
        if abs(lu - log_a) <= margin * max(1.0, abs(log_a)):
            ambiguous.append(b)
        if not lu < log_a or g in taken:
            continue
        taken.add(g)
        if K >= K_max:
            continue
        C[K] = C[idx[g]] + u
        idx[g] = K
        K += 1
        accepted.append(b)
    return {"C": C, "K": K, "idx": idx, "accepted": accepted, "ambiguous": ambiguous}


def merge(C: np.ndarray, K: int, idx: np.ndarray, lam: float, eps_split: float, eps_merge: float, B: int,
          step: int, seed: int, margin: float = 1e-5) -> Dict:
    """One batched merge step (see the module docstring).  Returns the new C,
    K, idx, the surviving merges [(c, c')], and ambiguous proposals."""
    C = np.array(C, np.float64)
    idx = np.array(idx, np.int64)
    if K < 2:
        return {"C": C, "K": K, "idx": idx, "merges": [], "ambiguous": []}
    named, merges, ambiguous = set(), [], []
    for b in range(B):
        w = _words(16 * b, MERGE_TAG, step, seed)
        c = choice(w[0], K)
        c2 = choice(w[1], K - 1)
        c2 += int(c2 >= c)
        d2 = float(np.sum((C[c] - C[c2]) ** 2))
        log_a = min(0.0, lam + log_q_sm(d2, eps_split, eps_merge))
        t = -d2 / (2.0 * eps_merge ** 2) + log_a
        lu = math.log(float(uniform24(w[2])))
        if abs(lu - t) <= margin * max(1.0, abs(t)):
            ambiguous.append(b)
        if not lu < t:
            continue
        if c not in named and c2 not in named:
            merges.append((c, c2))
        named.update((c, c2))
    remap = np.arange(K)
    freed = np.zeros(K, bool)
    for c, c2 in merges:
        remap[c2] = c
        freed[c2] = True
    K2 = K - len(merges)
    holes = [r for r in range(K2) if freed[r]]
    movers = [r for r in range(K2, K) if not freed[r]]
    assert len(holes) == len(movers)
    move = np.arange(K)
    for h, m in zip(holes, movers):
        C[h] = C[m]
        move[m] = h
    final = move[remap]
    idx = final[idx]
    return {"C": C, "K": K2, "idx": idx, "merges": merges, "ambiguous": ambiguous}
