"""Oracle for the simplified DP problem (S-DP) of the paper's Section II.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``): the tests,
the smoke check and the benchmark's CPU-baseline leg are its only callers,
and it shares no code with the GPU library.

Definition 1 (Section II-A): a one-dimensional solution table ST[0..n-1],
offsets a_1 > a_2 > ... > a_k > 0 and a semigroup operator; ST[0..a_1-1] are
preset and every later element is the operator folded over the elements
a_j places before it, Eq. (1):

    ST[i] = ST[i - a_1] (x) ST[i - a_2] (x) ... (x) ST[i - a_k],   i >= a_1.

:func:`solve` is that definition in the order of the sequential algorithm of
Fig. 1 (i ascending, j ascending), on int32 values with three operators:
minimum (the one the paper measures, Table I), maximum, and addition
modulo 2^32.  :func:`pipeline` runs the pipeline algorithm of Fig. 2 step by
step in lockstep (thread j updates ST[i - j + 1] from ST[i - j + 1 - a_j]),
for small inputs, as a reading of that figure.
"""
from __future__ import annotations

import numpy as np

OPS = ("min", "max", "add")


def _fold(op: str, vals: np.ndarray):
    if op == "min":
        return vals.min()
    if op == "max":
        return vals.max()
    if op == "add":
        return np.uint32(vals.astype(np.uint32).sum(dtype=np.uint64) & 0xFFFFFFFF).view(np.int32)
    raise ValueError(op)


def check(offsets, n: int) -> None:
    """Raises ValueError unless the offsets meet Definition 1 and fit n."""
    a = np.asarray(offsets, dtype=np.int64)
    if a.ndim != 1 or a.size < 1:
        raise ValueError("need k >= 1 offsets")
    if np.any(a[1:] >= a[:-1]) or a[-1] < 1:
        raise ValueError("offsets must be strictly decreasing and positive")
    if n < 1 or a[0] > n:
        raise ValueError("need 1 <= a_1 <= n")


def solve(offsets, init, n: int, op: str = "min") -> np.ndarray:
    """ST[0..n-1] (int32) by Eq. (1); init holds ST[0..a_1-1]."""
    check(offsets, n)
    a = np.asarray(offsets, dtype=np.int64)
    st = np.zeros(n, dtype=np.int32)
    st[:a[0]] = np.asarray(init, dtype=np.int32)[:a[0]]
    for i in range(int(a[0]), n):
        st[i] = _fold(op, st[i - a])
    return st


def _combine(op: str, x, y):
    if op == "min":
        return min(x, y)
    if op == "max":
        return max(x, y)
    return (x + y) & 0xFFFFFFFF


def pipeline(offsets, init, n: int, op: str = "min"):
    """Fig. 2 run in lockstep: returns (ST as int32 array, number of steps).

    In each step every active thread j (a_1 <= i - j + 1 < n) reads
    ST[i_j - a_j] as it was before the step, then all write.  Values are
    kept as Python ints (addition taken modulo 2^32).
    """
    check(offsets, n)
    a = [int(x) for x in offsets]
    k = len(a)
    st = [int(x) & 0xFFFFFFFF if op == "add" else int(x) for x in list(init)[:a[0]]]
    st += [0] * (n - a[0])
    steps = 0
    for i in range(a[0], n + k - 1):
        reads = []
        for j in range(1, k + 1):
            ij = i - j + 1
            if a[0] <= ij < n:
                reads.append((j, ij, st[ij - a[j - 1]]))
        for j, ij, v in reads:
            st[ij] = v if j == 1 else _combine(op, st[ij], v)
        steps += 1
    out = np.array([(x - (1 << 32)) if op == "add" and x >= (1 << 31) else x for x in st],
                   dtype=np.int64).astype(np.int32)
    return out, steps
