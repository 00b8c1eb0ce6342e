"""Pins for the optimal-BST oracle (no GPU): the textbook's worked example,
brute force over every BST of small key sets (cost counted from node
depths), the smallest-root tie rule, and the table layout."""
import random

import numpy as np
import pytest

from oracle import interval


def test_textbook_example():
    # Cormen et al., Introduction to Algorithms, Section 15.5 (Fig. 15.9):
    # five keys, weights in hundredths; expected cost 2.75, root k_2.
    p = [15, 10, 5, 10, 20]
    q = [5, 10, 5, 5, 5, 10]
    e, root = interval.optimal_bst(p, q)
    assert e[(1, 5)] == 275 and root[(1, 5)] == 2
    assert e[(1, 0)] == 5 and e[(6, 5)] == 10


def _tree_from_root(root, i, j):
    if i > j:
        return None
    r = root[(i, j)]
    return (_tree_from_root(root, i, r - 1), r, _tree_from_root(root, r + 1, j))


@pytest.mark.parametrize("seed", range(30))
def test_brute_force(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 6)
    hi = rng.choice([1, 3, 20, 1000])
    p = [rng.randint(0, hi) for _ in range(n)]
    q = [rng.randint(0, hi) for _ in range(n + 1)]
    e, root = interval.optimal_bst(p, q)
    trees = interval.all_trees(1, n)
    costs = [interval.search_cost(t, p, q) for t in trees]
    assert e[(1, n)] == min(costs)
    assert interval.search_cost(_tree_from_root(root, 1, n), p, q) == e[(1, n)]
    # smallest optimal root
    best_root = min(t[1] for t, c in zip(trees, costs) if c == min(costs))
    assert root[(1, n)] == best_root


def test_table_layout():
    rng = np.random.default_rng(3)
    n = 9
    p = rng.integers(0, 50, size=n)
    q = rng.integers(0, 50, size=n + 1)
    E, R = interval.obst_tables(p, q)
    assert np.array_equal(E, E.T)
    assert np.array_equal(np.diag(E), q)
    e, root = interval.optimal_bst(p, q)
    for a in range(n + 1):
        for b in range(a + 1, n + 1):
            assert E[a][b] == e[(a + 1, b)] and R[a][b] == root[(a + 1, b)]
            assert a + 1 <= R[a][b] <= b
    assert np.all(R[np.tril_indices(n + 1)] == -1)


def test_zero_key_weights_only_gaps_count():
    # With every p = 0 the cost is the sum over gaps of (depth + 1) q; with
    # a single weighted gap the optimal tree puts it as shallow as it can.
    # An end gap can hang off the root (depth 1: root k_1 or k_n); an inner
    # gap d_g sits below two keys at least (root k_g, then k_g+1): depth 2.
    n = 6
    for g in range(n + 1):
        q = [0] * (n + 1)
        q[g] = 7
        e, _ = interval.optimal_bst([0] * n, q)
        assert e[(1, n)] == (2 if g in (0, n) else 3) * 7


@pytest.mark.parametrize("seed", range(12))
def test_by_length_form_equals_textbook_loops(seed):
    # The numpy by-length form (used for inputs too large for the loops)
    # against the textbook loops, which the brute force above pins; ties
    # (small weights) included.
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(0, 45))
    hi = int(rng.choice([0, 1, 3, 1000, 1 << 20]))
    p = rng.integers(0, hi + 1, size=n)
    q = rng.integers(0, hi + 1, size=n + 1)
    E, R = interval.obst_tables(p, q)
    E2, R2 = interval.obst_tables_by_length(p, q)
    assert E2.dtype == E.dtype and R2.dtype == R.dtype
    assert np.array_equal(E, E2) and np.array_equal(R, R2)
