"""Oracle for other interval DPs solved by the same split recurrence.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``): the tests,
the smoke check and the benchmark's CPU-baseline leg are its only callers,
and it shares no code with the GPU library.

The paper closes Section IV by proposing to carry its technique to more
general DP problems.  The optimal binary search tree is the textbook's
other interval DP of this shape (the same reference the paper takes MCM
from): keys k_1 < ... < k_n searched with weights p_1..p_n, gaps d_0..d_n
(unsuccessful searches) with weights q_0..q_n, and

    e[i][i-1] = q_{i-1}
    e[i][j]   = min over i <= r <= j of e[i][r-1] + e[r+1][j] + w(i, j)
    w(i, j)   = p_i + ... + p_j + q_{i-1} + ... + q_j

:func:`optimal_bst` is that recurrence in the textbook's own 1-based
notation (integer weights, exact), smallest root on ties.
:func:`search_cost` prices a given tree directly from node depths, for
brute-force pins.
"""
from __future__ import annotations

import numpy as np


def optimal_bst(p, q):
    """(e, root) as dicts keyed (i, j), 1 <= i <= n+1, i-1 <= j <= n.

    p: n key weights (p[0] is p_1), q: n+1 gap weights (q[0] is q_0).
    root[(i, j)] is the smallest optimal root r for keys i..j (j >= i).
    """
    n = len(p)
    if len(q) != n + 1:
        raise ValueError("need n+1 gap weights")
    P = [0] + [int(x) for x in p]          # P[i] = p_i
    Q = [int(x) for x in q]                # Q[i] = q_i
    e, w, root = {}, {}, {}
    for i in range(1, n + 2):
        e[(i, i - 1)] = Q[i - 1]
        w[(i, i - 1)] = Q[i - 1]
    for length in range(1, n + 1):
        for i in range(1, n - length + 2):
            j = i + length - 1
            w[(i, j)] = w[(i, j - 1)] + P[j] + Q[j]
            best, arg = None, None
            for r in range(i, j + 1):
                t = e[(i, r - 1)] + e[(r + 1, j)] + w[(i, j)]
                if best is None or t < best:
                    best, arg = t, r
            e[(i, j)] = best
            root[(i, j)] = arg
    return e, root


def search_cost(tree, p, q) -> int:
    """Expected-cost numerator of a BST given as nested (left, key, right)
    tuples over keys 1..n, with None for a gap: sum of (depth + 1) times
    the weight of every key and every gap (gaps numbered left to right)."""
    total = 0
    gap = 0

    def walk(node, depth):
        nonlocal total, gap
        if node is None:
            total += (depth + 1) * int(q[gap])
            gap += 1
            return
        left, key, right = node
        walk(left, depth + 1)
        total += (depth + 1) * int(p[key - 1])
        walk(right, depth + 1)

    walk(tree, 0)
    return total


def all_trees(lo: int, hi: int):
    """Every BST over keys lo..hi (None when empty)."""
    if lo > hi:
        return [None]
    out = []
    for r in range(lo, hi + 1):
        for left in all_trees(lo, r - 1):
            for right in all_trees(r + 1, hi):
                out.append((left, r, right))
    return out


def obst_tables_by_length(p, q):
    """obst_tables computed with numpy, one interval length at a time: the
    same textbook recurrence (w(i, j) = w(i, j-1) + p_j + q_j; e(i, j) the
    minimum over roots r of e(i, r-1) + e(r+1, j), plus w(i, j); the first
    minimum, i.e. the smallest root), each length's cells and roots formed
    as one array, for inputs too large for the pure-Python loops.  Same
    return layout as obst_tables."""
    n = len(p)
    if len(q) != n + 1:
        raise ValueError("need n+1 gap weights")
    P = np.concatenate([[0], np.asarray(p, dtype=np.int64)])   # P[i] = p_i
    Q = np.asarray(q, dtype=np.int64)                           # Q[i] = q_i
    # E[i][j] holds the textbook e(i, j) for 1 <= i <= n+1, i-1 <= j <= n.
    E = np.zeros((n + 2, n + 1), dtype=np.int64)
    W = np.zeros((n + 2, n + 1), dtype=np.int64)
    R = np.zeros((n + 2, n + 1), dtype=np.int64)
    idx = np.arange(1, n + 2)
    E[idx, idx - 1] = Q[idx - 1]
    W[idx, idx - 1] = Q[idx - 1]
    for length in range(1, n + 1):
        i = np.arange(1, n - length + 2)            # every cell of this length
        j = i + length - 1
        W[i, j] = W[i, j - 1] + P[j] + Q[j]
        r = i[:, None] + np.arange(length)[None, :]  # roots i..j per cell
        cand = E[i[:, None], r - 1] + E[r + 1, j[:, None]]
        k = np.argmin(cand, axis=1)                   # first minimum: smallest root
        E[i, j] = cand[np.arange(i.size), k] + W[i, j]
        R[i, j] = i + k
    L = n + 1
    Et = np.zeros((L, L), dtype=np.int64)
    Rt = np.full((L, L), -1, dtype=np.int32)
    for a in range(L):
        b = np.arange(a, L)
        Et[a, b] = E[a + 1, b]
        Et[b, a] = E[a + 1, b]
        Rt[a, b[1:]] = R[a + 1, b[1:]]
    return Et, Rt


def obst_tables(p, q):
    """The (n+1) x (n+1) int64 / int32 tables of the library's layout: gaps
    0..n as leaves; for a <= b, e[a][b] = e(a+1, b) of the textbook (keys
    a+1..b; e[a][a] = q_a), mirrored below the diagonal; root[a][b] = the
    smallest optimal root key (1-based) for a < b, -1 for a >= b."""
    e, root = optimal_bst(p, q)
    L = len(p) + 1
    E = np.zeros((L, L), dtype=np.int64)
    R = np.full((L, L), -1, dtype=np.int32)
    for a in range(L):
        for b in range(a, L):
            E[a][b] = E[b][a] = e[(a + 1, b)]
            if a < b:
                R[a][b] = root[(a + 1, b)]
    return E, R
