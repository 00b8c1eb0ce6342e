"""Pins for the parenthesization oracle (no GPU).

The oracle reads the optimal product order back out of a split table.  It is
pinned against things other than itself: exhaustive enumeration of every
parenthesization (cost counted from matrix shapes of the parsed text), the
textbook's own worked example, closed forms for tables whose tree is known,
an independent parse of its text, and the behaviour on tables that are not
split tables.
"""
import random

import numpy as np
import pytest

import oracle
from oracle import paren


def _parse(text):
    """Independent reading of a parenthesized product.

    Returns (nodes, root): nodes maps split k -> (lo, hi) of the product
    whose left operand ends at matrix k; root is the (lo, hi) of the whole.
    """
    stack = []  # entries: (lo, hi) of finished operands; "(" markers
    nodes = {}
    pos = 0
    while pos < len(text):
        c = text[pos]
        if c == "(":
            stack.append("(")
            pos += 1
        elif c == "A":
            end = pos + 1
            while end < len(text) and text[end].isdigit():
                end += 1
            t = int(text[pos + 1:end])
            stack.append((t, t))
            pos = end
        elif c == ")":
            right = stack.pop()
            left = stack.pop()
            assert stack.pop() == "(", "unbalanced text"
            assert left[1] + 1 == right[0], "operands not adjacent"
            nodes[left[1]] = (left[0], right[1])
            stack.append((left[0], right[1]))
            pos += 1
        else:
            raise AssertionError("unexpected character %r" % c)
    assert len(stack) == 1
    return nodes, stack[0]


def _shape_cost(text, p):
    """Scalar multiplications of evaluating the text, from matrix shapes."""
    stack = []
    pos = 0
    while pos < len(text):
        c = text[pos]
        if c == "(":
            stack.append("(")
            pos += 1
        elif c == "A":
            end = pos + 1
            while end < len(text) and text[end].isdigit():
                end += 1
            t = int(text[pos + 1:end])
            stack.append((int(p[t]), int(p[t + 1]), 0))
            pos = end
        else:
            r = stack.pop()
            l = stack.pop()
            stack.pop()
            assert l[1] == r[0], "non-conformable product"
            stack.append((l[0], r[1], l[2] + r[2] + l[0] * l[1] * r[1]))
            pos += 1
    return stack[0][2]


def _all_texts(i, j):
    if i == j:
        return ["A%d" % i]
    return ["(" + a + b + ")" for k in range(i, j)
            for a in _all_texts(i, k) for b in _all_texts(k + 1, j)]


def test_textbook_worked_example():
    # The six-matrix example of the textbook's matrix-chain section
    # (Cormen, Leiserson, Rivest, Stein, Introduction to Algorithms,
    # Section 15.2; 1-based there): optimal cost 15125 with the order
    # ((A1(A2A3))((A4A5)A6)).
    p = [30, 35, 15, 5, 10, 20, 25]
    m, s = oracle.fill(p)
    lo, hi, cost, text = paren.reconstruct(p, s)
    assert cost == 15125 == m[0][5]
    assert text == "((A0(A1A2))((A3A4)A5))"
    # Nodes by split: 0 -> A0(A1A2) = [0,2], 1 -> A1A2, 2 -> the root,
    # 3 -> A3A4, 4 -> (A3A4)A5.
    assert list(lo) == [0, 1, 0, 3, 3] and list(hi) == [2, 2, 5, 4, 5]


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_optimal_order(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 7)
    hi_dim = rng.choice([3, 12, 60])
    p = [rng.randint(1, hi_dim) for _ in range(n + 1)]
    m, s = oracle.fill(p)
    lo, hi, cost, text = paren.reconstruct(p, s)
    best = min(_shape_cost(t, p) for t in _all_texts(0, n - 1))
    assert _shape_cost(text, p) == best == cost
    assert len(text) == paren.parens_length(n)
    if n >= 2:
        nodes, root = _parse(text)
        assert root == (0, n - 1)
        assert sorted(nodes) == list(range(n - 1))
        for k in range(n - 1):
            assert nodes[k] == (lo[k], hi[k])
            assert s[lo[k]][hi[k]] == k


def test_equal_dims_right_deep():
    # Every split ties; the smallest split peels off the first matrix.
    n, d = 9, 7
    p = [d] * (n + 1)
    m, s = oracle.fill(p)
    lo, hi, cost, text = paren.reconstruct(p, s)
    assert text == "(A0(A1(A2(A3(A4(A5(A6(A7A8))))))))"
    assert list(lo) == list(range(n - 1)) and list(hi) == [n - 1] * (n - 1)
    assert cost == (n - 1) * d ** 3 == m[0][n - 1]


def _table(n, split):
    s = np.full((n, n), -1, dtype=np.int32)
    for i in range(n):
        for j in range(i + 1, n):
            s[i][j] = split(i, j)
    return s


def test_left_deep_table():
    n = 12
    s = _table(n, lambda i, j: j - 1)
    lo, hi, ok = paren.tree_from_splits(s, n)
    assert ok and lo == [0] * (n - 1) and hi == list(range(1, n))
    assert paren.parens_text(s, 4) == "(((A0A1)A2)A3)"


def test_balanced_table():
    n = 8
    s = _table(n, lambda i, j: (i + j) // 2)
    text = paren.parens_text(s, n)
    assert text == "(((A0A1)(A2A3))((A4A5)(A6A7)))"
    p = list(range(1, n + 2))
    lo, hi, cost, _ = paren.reconstruct(p, s)
    assert cost == _shape_cost(text, p)


@pytest.mark.parametrize("seed", range(20))
def test_random_split_tables_parse_back(seed):
    # Any table of valid splits defines one tree; its text parses back to
    # the same node intervals, whatever the dims.
    rng = random.Random(100 + seed)
    n = rng.randint(2, 60)
    s = _table(n, lambda i, j: rng.randint(i, j - 1))
    p = [rng.randint(1, 50) for _ in range(n + 1)]
    lo, hi, cost, text = paren.reconstruct(p, s)
    nodes, root = _parse(text)
    assert root == (0, n - 1)
    assert {k: (lo[k], hi[k]) for k in range(n - 1)} == nodes
    assert cost == _shape_cost(text, p)
    assert len(text) == paren.parens_length(n)


def test_single_matrix():
    lo, hi, cost, text = paren.reconstruct([4, 9], np.full((1, 1), -1, dtype=np.int32))
    assert len(lo) == 0 and cost == 0 and text == "A0"
    assert paren.parens_length(1) == 2


def test_length_closed_form():
    for n in (1, 2, 9, 10, 11, 99, 100, 101, 1234):
        digits = sum(len(str(t)) for t in range(n))
        assert paren.parens_length(n) == 2 * (n - 1) + n + digits


def test_not_a_split_table():
    n = 6
    s = _table(n, lambda i, j: i)
    s[0][n - 1] = n - 1          # the root's entry is out of range
    lo, hi, cost, text = paren.reconstruct(list(range(1, n + 2)), s)
    assert all(v == -1 for v in lo) and cost == -1 and text == ""
    s = _table(n, lambda i, j: i)
    s[2][5] = 1                  # below the root: [2,5] is reached, entry < i
    lo, hi, ok = paren.tree_from_splits(s, n)
    assert not ok
    # [0,5] -> k=0 ([1,5]) -> k=1 ([2,5]) stops; the rest stay -1
    assert lo == [0, 1, -1, -1, -1] and hi == [5, 5, -1, -1, -1]
