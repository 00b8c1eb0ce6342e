"""Seeded synthetic inputs for the matrix-chain solver.

This module holds random-number plumbing only -- none of the method's
arithmetic -- so both the GPU path and the CPU oracle can be fed from it.
The paper measures its MCM method on no dataset (its MCM evaluation is left
to future work), so every workload is synthetic.  All draws use NumPy's
PCG64 ``default_rng(seed)`` and ``integers(lo, hi, size, endpoint=True)``
(both bounds inclusive), in the order listed in each function.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def uniform_dims(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Dimension vector p[0..n] with iid integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=n + 1, endpoint=True, dtype=np.int32)


def single_n128() -> np.ndarray:
    """n = 128 matrices, dims uniform in [1, 64], seed 0."""
    return uniform_dims(128, 1, 64, 0)


def single_n2048() -> np.ndarray:
    """n = 2048 matrices, dims uniform in [1, 1024], seed 1."""
    return uniform_dims(2048, 1, 1024, 1)


def single_n8192() -> np.ndarray:
    """n = 8192 matrices, dims uniform in [1, 1024], seed 2."""
    return uniform_dims(8192, 1, 1024, 2)


@dataclass
class Batch:
    """A batch of chains: ns[b] matrices each, dims concatenated."""
    ns: np.ndarray        # int32[count]
    p_off: np.ndarray     # int64[count]: start of chain b's dims in p_all
    p_all: np.ndarray     # int32[sum(ns + 1)]

    def dims(self, b: int) -> np.ndarray:
        o = int(self.p_off[b])
        return self.p_all[o:o + int(self.ns[b]) + 1]


def make_batch(chains) -> Batch:
    """Pack a list of dimension vectors into a :class:`Batch`."""
    chains = [np.asarray(c, dtype=np.int32) for c in chains]
    ns = np.array([c.size - 1 for c in chains], dtype=np.int32)
    p_off = np.zeros(len(chains), dtype=np.int64)
    if len(chains) > 1:
        p_off[1:] = np.cumsum([c.size for c in chains[:-1]])
    p_all = np.concatenate(chains) if chains else np.zeros(0, dtype=np.int32)
    return Batch(ns=ns, p_off=p_off, p_all=p_all.astype(np.int32))


def batched_4096(count: int = 4096, seed: int = 3, n_lo: int = 16, n_hi: int = 512,
                 p_hi: int = 256) -> Batch:
    """Batch of `count` chains: n_b uniform in [n_lo, n_hi], then per chain,
    in order, dims uniform in [1, p_hi] (defaults: 4096 chains, seed 3)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi, size=count, endpoint=True, dtype=np.int32)
    chains = [rng.integers(1, p_hi, size=int(nb) + 1, endpoint=True, dtype=np.int32)
              for nb in ns]
    return make_batch(chains)


@dataclass
class RequestStream:
    """Open-loop request stream: arrival offsets (s) and one chain each."""
    arrivals: np.ndarray  # float64[count], seconds from stream start
    batch: Batch


def serving_stream(count: int = 20000, rate: float = 1000.0, seed: int = 4,
                   n_lo: int = 8, n_hi: int = 4096, p_hi: int = 1024) -> RequestStream:
    """Poisson arrivals at `rate` requests/s; n log-uniform in [n_lo, n_hi]
    (rounded); dims uniform in [1, p_hi].  Draw order: all gaps, all n,
    then each request's dims."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(np.int32)
    ns = np.clip(ns, n_lo, n_hi)
    chains = [rng.integers(1, p_hi, size=int(nb) + 1, endpoint=True, dtype=np.int32)
              for nb in ns]
    return RequestStream(arrivals=np.cumsum(gaps), batch=make_batch(chains))


# Structured chains for edge cases and counters.

def all_equal(n: int, d: int) -> np.ndarray:
    return np.full(n + 1, d, dtype=np.int32)


def increasing(n: int, lo: int = 1) -> np.ndarray:
    return np.arange(lo, lo + n + 1, dtype=np.int32)


def decreasing(n: int, lo: int = 1) -> np.ndarray:
    return increasing(n, lo)[::-1].copy()


def alternating(n: int, a: int = 1, b: int = 1024) -> np.ndarray:
    return np.where(np.arange(n + 1) % 2 == 0, a, b).astype(np.int32)


def tie_heavy(n: int, seed: int) -> np.ndarray:
    """Dims drawn from {1, 2}: many equal-cost splits."""
    return uniform_dims(n, 1, 2, seed)


SPLIT_SHAPES = ("left", "right", "balanced", "zigzag", "random")


def split_table(n: int, shape: str, seed: int = 0) -> np.ndarray:
    """An n x n int32 table of valid splits (i <= s[i][j] < j above the
    diagonal, -1 elsewhere) whose tree has a chosen shape, as input for
    reading a tree back from a table:

    left      s[i][j] = j-1: one long chain of left children
    right     s[i][j] = i: one long chain of right children
    balanced  s[i][j] = (i+j)//2
    zigzag    alternates j-1 and i along the path from the root, so every
              step of the path changes direction
    random    iid uniform in [i, j-1] (PCG64 ``random`` doubles, row-major)
    """
    i = np.arange(n, dtype=np.int64)[:, None]
    j = np.arange(n, dtype=np.int64)[None, :]
    if shape == "left":
        s = np.broadcast_to(j - 1, (n, n))
    elif shape == "right":
        s = np.broadcast_to(i, (n, n))
    elif shape == "balanced":
        s = (i + j) // 2
    elif shape == "zigzag":
        s = np.where((i + (n - 1 - j)) % 2 == 0, j - 1, i)
    elif shape == "random":
        u = np.random.default_rng(seed).random((n, n))
        s = i + np.floor(u * np.maximum(j - i, 0)).astype(np.int64)
    else:
        raise ValueError(shape)
    return np.where(j > i, s, -1).astype(np.int32)


# Simplified DP (S-DP) inputs.  The paper's Table I gives n and k ranges
# only; each configuration here takes the top of a range.
SDP_CONFIGS = {
    "sdp_small": (1 << 15, 1 << 13),
    "sdp_medium": (1 << 17, 1 << 15),
    "sdp_large": (1 << 19, 1 << 17),
}


def sdp_instance(n: int, k: int, seed: int, kind: str = "random"):
    """(offsets, init) for an S-DP table of n elements with k offsets.

    random       k distinct offsets drawn without replacement from [1, 2k]
                 (``choice(2k, k, replace=False) + 1``), sorted descending
    consecutive  k, k-1, ..., 1 (the worst case of Fig. 4)
    init: the a_1 preset values, iid in [0, 2^30) (drawn after the offsets).
    """
    rng = np.random.default_rng(seed)
    if kind == "random":
        a = np.sort(rng.choice(2 * k, size=k, replace=False) + 1)[::-1]
    elif kind == "consecutive":
        a = np.arange(k, 0, -1)
    else:
        raise ValueError(kind)
    a = np.ascontiguousarray(a, dtype=np.int32)
    init = rng.integers(0, 1 << 30, size=int(a[0]), dtype=np.int32)
    return a, init
