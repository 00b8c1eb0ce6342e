"""The MCM table in the paper's own formulation (pure Python, small n).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section IV of the paper lines the triangular solution table up into a 1-D
array ``ST`` in the order its elements are computed, diagonal by diagonal
(Fig. 5 and Fig. 7): for n matrices there are n(n+1)/2 elements, and the
first n -- the main diagonal -- are preset.  Every other element is
Eq. (2): ``ST[x]`` is the smaller-operand operator folded over its k_x
operand pairs ``f(l_(x,j), r_(x,j))``, with k_x <= n-1.

Indices here are 1-based, as in the paper: element (a, b) of the table,
a <= b, covers matrices a..b, and matrix t has p[t-1] rows and p[t]
columns.  Split j of element (a, b) joins (a, a+j-1) and (a+j, b); the
paper leaves f to the textbook MCM definition, which adds the two
sub-results and the cost p[a-1] * p[a+j-1] * p[b] of the final product.
The fold keeps the running value when a later operand is equal (the
operator returns the smaller operand; an equal one is not smaller), so the
recorded split is the smallest j attaining the minimum.

This module is written for reading, not speed: O(n^3) Python loops.
"""
from __future__ import annotations

import numpy as np


def element_index(a: int, b: int, n: int) -> int:
    """1-based position in ST of table element (a, b), 1 <= a <= b <= n.

    Diagonal d = b - a holds n - d elements; diagonals are laid out in
    increasing d, each top row first (Fig. 5 numbering).
    """
    if not (1 <= a <= b <= n):
        raise ValueError("need 1 <= a <= b <= n")
    d = b - a
    before = sum(n - e for e in range(d))  # elements on diagonals 0..d-1
    return before + a


def element_at(x: int, n: int) -> tuple[int, int]:
    """Inverse of :func:`element_index`: ST position x -> (a, b)."""
    total = n * (n + 1) // 2
    if not (1 <= x <= total):
        raise ValueError("position out of range")
    d = 0
    while x > n - d:
        x -= n - d
        d += 1
    return x, x + d


def operand_pairs(x: int, n: int) -> list[tuple[int, int]]:
    """The pairs (l_(x,j), r_(x,j)), j = 1..k_x, of Eq. (2) for element x."""
    a, b = element_at(x, n)
    return [(element_index(a, a + j - 1, n), element_index(a + j, b, n))
            for j in range(1, b - a + 1)]


def solve_linear(p) -> tuple[list[int], list[int]]:
    """Fill ST in linear order by Eq. (2); return (ST, SPLIT), 1-based lists.

    ST[x] is the optimal cost of element x; SPLIT[x] is the 1-based matrix
    index after which the winning split cuts (a+j-1 for split j), 0 on the
    main diagonal.  Index 0 of both lists is unused.
    """
    p = [int(v) for v in p]
    n = len(p) - 1
    if n < 1 or min(p) < 1:
        raise ValueError("invalid chain")
    total = n * (n + 1) // 2
    ST = [0] * (total + 1)
    SPLIT = [0] * (total + 1)
    # ST[1..n] are the preset main-diagonal elements (cost 0).
    for x in range(n + 1, total + 1):
        a, b = element_at(x, n)
        best = None
        best_split = 0
        for j, (l, r) in enumerate(operand_pairs(x, n), start=1):
            v = ST[l] + ST[r] + p[a - 1] * p[a + j - 1] * p[b]   # f(l, r)
            if best is None or v < best:                         # the fold
                best = v
                best_split = a + j - 1
        ST[x] = best
        SPLIT[x] = best_split
    return ST, SPLIT


def solve_tables(p) -> tuple[np.ndarray, np.ndarray]:
    """ST unfolded into the library's 0-based n x n output contract.

    m[i][j] = m[j][i] = ST of element (i+1, j+1); s[i][j] = 0-based split
    k (between matrices k and k+1, 0-based) for i < j, and -1 for i >= j.
    """
    ST, SPLIT = solve_linear(p)
    n = len(p) - 1
    m = np.zeros((n, n), dtype=np.int64)
    s = np.full((n, n), -1, dtype=np.int32)
    for x in range(1, len(ST)):
        a, b = element_at(x, n)
        m[a - 1, b - 1] = m[b - 1, a - 1] = ST[x]
        if a < b:
            s[a - 1, b - 1] = SPLIT[x] - 1
    return m, s
