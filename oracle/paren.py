"""Oracle for reading the optimal parenthesization back out of a split table.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``): the tests,
the smoke check and the benchmark's CPU-baseline leg are its only callers,
and it shares no code with the GPU library.

The paper takes the MCM problem and its table from the textbook formulation
it cites in Section IV; there the optimal order is recovered from the split
table by recursion: the product of matrices i..j is the product of the
results for i..s[i][j] and s[i][j]+1..j, down to single matrices.  Written
out here with an explicit stack, in plain Python:

* every internal node of the tree is named by its split k (0 <= k < n-1):
  the node multiplies (A_lo..A_k) by (A_k+1..A_hi), and ``lo[k]``, ``hi[k]``
  record that interval;
* the tree's cost is the sum over its nodes of p[lo] * p[k+1] * p[hi+1];
* the text is the fully parenthesized product, matrices written ``A<t>``
  (0-based), e.g. ``((A0A1)A2)``; a single matrix is ``A0``.

A table entry that is not a split of its cell (s[i][j] outside [i, j-1])
is reported rather than followed: the subtree below that cell is left out,
``lo``/``hi`` of its splits stay -1, the cost is -1 and the text is empty.
"""
from __future__ import annotations

import numpy as np


def tree_from_splits(s, n: int):
    """(lo, hi, ok): the node interval of every split, top-down from [0, n-1].

    ``s`` is indexable as s[i][j] (an n x n table, row-major semantics).
    ``lo``/``hi`` are int lists of n-1 entries, -1 where not reached; ``ok``
    is False when some reached cell holds an entry that is not a split.
    """
    lo = [-1] * max(n - 1, 0)
    hi = [-1] * max(n - 1, 0)
    ok = True
    stack = [(0, n - 1)] if n >= 2 else []
    while stack:
        i, j = stack.pop()
        k = int(s[i][j])
        if not (i <= k < j):
            ok = False
            continue
        lo[k], hi[k] = i, j
        if i < k:
            stack.append((i, k))
        if k + 1 < j:
            stack.append((k + 1, j))
    return lo, hi, ok


def tree_cost(p, lo, hi, ok: bool = True) -> int:
    """Scalar multiplications of the tree (lo, hi); -1 when ``ok`` is False."""
    if not ok:
        return -1
    total = 0
    for k in range(len(lo)):
        total += int(p[lo[k]]) * int(p[k + 1]) * int(p[hi[k] + 1])
    return total


def parens_text(s, n: int) -> str:
    """The parenthesized product, built by the textbook's recursion on s.

    Empty when the walk meets an entry that is not a split.
    """
    out = []
    # Work items: ("cell", i, j) expands a sub-chain, ("text", str) emits.
    work = [("cell", 0, n - 1)]
    while work:
        item = work.pop()
        if item[0] == "text":
            out.append(item[1])
            continue
        _, i, j = item
        if i == j:
            out.append("A%d" % i)
            continue
        k = int(s[i][j])
        if not (i <= k < j):
            return ""
        # Pushed in reverse so they pop as "(", left, right, ")".
        work.append(("text", ")"))
        work.append(("cell", k + 1, j))
        work.append(("cell", i, k))
        work.append(("text", "("))
    return "".join(out)


def parens_length(n: int) -> int:
    """Characters in the text of any full parenthesization of n matrices.

    Each of the n-1 products adds one "(" and one ")"; matrix t adds "A" and
    the decimal digits of t.
    """
    return 2 * (n - 1) + sum(1 + len(str(t)) for t in range(n))


def reconstruct(p, s):
    """Everything at once for a chain p[0..n] and its split table s.

    Returns (lo int32[n-1], hi int32[n-1], cost int, text str).
    """
    n = len(p) - 1
    lo, hi, ok = tree_from_splits(s, n)
    return (np.asarray(lo, dtype=np.int32), np.asarray(hi, dtype=np.int32),
            tree_cost(p, lo, hi, ok), parens_text(s, n) if ok else "")
