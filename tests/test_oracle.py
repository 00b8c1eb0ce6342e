"""Pins for the CPU oracle (no GPU).

The oracle is only trusted once it agrees with things other than itself:
brute-force enumeration of every parenthesization (with the cost of a tree
counted from matrix shapes, not from the recurrence), closed forms,
invariants, optimal substructure on windows, and the paper's worked n=5
indexing example.  Each pin is chosen so a plausible slip in the oracle
(a wrong dimension index, <= instead of <, a dropped term, a transposed
operand) fails at least one of them.
"""
import os
import random

import numpy as np
import pytest

import oracle
from oracle import linear
from paper_2008_01938_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Brute force: every full parenthesization, cost counted from matrix shapes.
# --------------------------------------------------------------------------

def _trees(i, j):
    """All full binary trees over matrices i..j (0-based), as nested tuples."""
    if i == j:
        return [i]
    out = []
    for k in range(i, j):
        for left in _trees(i, k):
            for right in _trees(k + 1, j):
                out.append((left, right))
    return out


def _shape_cost(tree, p):
    """(rows, cols, scalar multiplications) of evaluating `tree`."""
    if isinstance(tree, int):
        return p[tree], p[tree + 1], 0
    lr, lc, lcost = _shape_cost(tree[0], p)
    rr, rc, rcost = _shape_cost(tree[1], p)
    assert lc == rr, "non-conformable product"
    return lr, rc, lcost + rcost + lr * lc * rc


def _root_split(tree):
    """Index of the last matrix of the root's left factor."""
    left = tree[0]
    while not isinstance(left, int):
        left = left[1]
    return left


def brute_force(p):
    """m, s by exhaustive enumeration for every sub-chain (n <= 9)."""
    p = [int(v) for v in p]
    n = len(p) - 1
    m = np.zeros((n, n), dtype=np.int64)
    s = np.full((n, n), -1, dtype=np.int32)
    for i in range(n):
        for j in range(i + 1, n):
            best, splits = None, []
            for t in _trees(i, j):
                c = _shape_cost(t, p)[2]
                if best is None or c < best:
                    best, splits = c, [_root_split(t)]
                elif c == best:
                    splits.append(_root_split(t))
            m[i, j] = m[j, i] = best
            s[i, j] = min(splits)
    return m, s


def test_brute_force_counts_trees():
    # Catalan numbers: 1, 1, 2, 5, 14, 42, 132 trees for 1..7 matrices.
    assert [len(_trees(0, k)) for k in range(7)] == [1, 1, 2, 5, 14, 42, 132]


@pytest.mark.parametrize("n", list(range(1, 10)))
def test_oracle_matches_brute_force_random(n):
    for seed in range(3):
        p = workloads.uniform_dims(n, 1, 40, 1000 * n + seed)
        bm, bs = brute_force(p)
        m, s = oracle.fill(p)
        np.testing.assert_array_equal(m, bm)
        np.testing.assert_array_equal(s, bs)


@pytest.mark.parametrize("n", [2, 3, 5, 7, 9])
def test_oracle_matches_brute_force_ties(n):
    # Dims in {1, 2} make many parenthesizations cost the same, which pins
    # the smallest-split tie rule.
    for seed in range(6):
        p = workloads.tie_heavy(n, 77 + seed)
        bm, bs = brute_force(p)
        m, s = oracle.fill(p)
        np.testing.assert_array_equal(m, bm)
        np.testing.assert_array_equal(s, bs)


@pytest.mark.parametrize("n", [1, 2, 4, 6, 8])
def test_linear_formulation_matches_brute_force(n):
    for seed in range(3):
        p = workloads.uniform_dims(n, 1, 9, 500 + seed)
        bm, bs = brute_force(p)
        m, s = linear.solve_tables(p)
        np.testing.assert_array_equal(m, bm)
        np.testing.assert_array_equal(s, bs)


def test_c_oracle_matches_linear_formulation():
    rng = random.Random(5)
    for _ in range(12):
        n = rng.randint(1, 28)
        p = workloads.uniform_dims(n, 1, rng.choice([2, 9, 300]), rng.randrange(10**6))
        m, s = oracle.fill(p)
        lm, ls = linear.solve_tables(p)
        np.testing.assert_array_equal(m, lm)
        np.testing.assert_array_equal(s, ls)


# --------------------------------------------------------------------------
# The paper's worked example: diagonal-order numbering and operand pairs.
# --------------------------------------------------------------------------

def _golden_operands():
    rows = []
    with open(os.path.join(GOLDEN, "paper_n5_operands.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, pairs = line.split(":")
            n, x = (int(v) for v in head.split())
            pl = [tuple(int(v) for v in pr.split()) for pr in pairs.split(",")]
            rows.append((n, x, pl))
    return rows


def test_paper_example_operand_pairs():
    rows = _golden_operands()
    assert len(rows) == 2
    for n, x, pairs in rows:
        assert linear.operand_pairs(x, n) == pairs


def test_paper_example_numbering_is_diagonal_order():
    n = 5
    # The first n elements are the preset main diagonal, then diagonal 1 ...
    assert [linear.element_index(a, a, n) for a in range(1, 6)] == [1, 2, 3, 4, 5]
    assert [linear.element_index(a, a + 1, n) for a in range(1, 5)] == [6, 7, 8, 9]
    assert linear.element_index(1, 5, n) == n * (n + 1) // 2
    for x in range(1, 16):
        assert linear.element_index(*linear.element_at(x, n), n) == x


# --------------------------------------------------------------------------
# Closed forms.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [1, 3, 64, 1024])
def test_closed_form_all_equal_dims(d):
    # Every split of (i, j) costs (j-i) d^3, so all tie and the smallest wins.
    n = 60
    m, s = oracle.fill(workloads.all_equal(n, d))
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    np.testing.assert_array_equal(m, np.abs(jj - ii).astype(np.int64) * d ** 3)
    np.testing.assert_array_equal(s, np.where(ii < jj, ii, -1))


def test_closed_form_two_matrices():
    for p in ([3, 5, 7], [1, 1, 1], [1000, 1, 1000]):
        m, s = oracle.fill(p)
        assert m[0, 1] == m[1, 0] == p[0] * p[1] * p[2]
        assert s.tolist() == [[-1, 0], [-1, -1]]


def test_single_matrix():
    m, s = oracle.fill([4, 9])
    assert m.tolist() == [[0]] and s.tolist() == [[-1]]


# --------------------------------------------------------------------------
# Invariants at a size brute force cannot reach.
# --------------------------------------------------------------------------

def _rebuild_cost(p, s, i, j):
    """Cost of the parenthesization encoded by s, counted from shapes."""
    if i == j:
        return 0
    k = int(s[i, j])
    return _rebuild_cost(p, s, i, k) + _rebuild_cost(p, s, k + 1, j) + \
        int(p[i]) * int(p[k + 1]) * int(p[j + 1])


@pytest.mark.parametrize("seed,pmax", [(11, 1024), (12, 64), (13, 2)])
def test_invariants(seed, pmax):
    n = 180
    p = workloads.uniform_dims(n, 1, pmax, seed)
    m, s = oracle.fill(p)
    pi = p.astype(np.int64)
    assert np.all(np.diag(m) == 0)
    np.testing.assert_array_equal(m, m.T)
    idx = np.arange(n - 1)
    np.testing.assert_array_equal(m[idx, idx + 1], pi[:-2] * pi[1:-1] * pi[2:])
    np.testing.assert_array_equal(s[idx, idx + 1], idx)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    upper = ii < jj
    assert np.all(s[~upper] == -1)
    assert np.all((s[upper] >= ii[upper]) & (s[upper] < jj[upper]))
    # m[i][j] is realised by its recorded split.
    iu, ju = ii[upper], jj[upper]
    ku = s[upper].astype(np.int64)
    np.testing.assert_array_equal(
        m[upper], m[iu, ku] + m[ku + 1, ju] + pi[iu] * pi[ku + 1] * pi[ju + 1])
    assert _rebuild_cost(p, s, 0, n - 1) == m[0, n - 1]
    # No split beats it (full recurrence re-check from the table itself).
    cells = np.stack([iu, ju], axis=1)
    assert oracle.check_cells(p, m, s, cells) == 0


def test_optimal_substructure_windows():
    # The table of a sub-chain is the matching block of the full table.
    n = 150
    p = workloads.uniform_dims(n, 1, 1024, 21)
    m, s = oracle.fill(p)
    for i0, L in [(0, 40), (37, 50), (100, 50), (149, 1)]:
        wm, ws = oracle.fill(p[i0:i0 + L + 1])
        np.testing.assert_array_equal(wm, m[i0:i0 + L, i0:i0 + L])
        shifted = np.where(ws >= 0, ws + i0, -1)
        np.testing.assert_array_equal(shifted, s[i0:i0 + L, i0:i0 + L])


def test_openmp_threads_agree():
    p = workloads.uniform_dims(300, 1, 1024, 31)
    m1, s1 = oracle.fill(p, threads=1)
    m4, s4 = oracle.fill(p, threads=4)
    np.testing.assert_array_equal(m1, m4)
    np.testing.assert_array_equal(s1, s4)


# --------------------------------------------------------------------------
# Validation and the cell checker.
# --------------------------------------------------------------------------

def test_validation():
    assert oracle.validate([5]) == oracle.INVALID           # n = 0
    assert oracle.validate([3, 0, 4]) == oracle.INVALID     # zero dimension
    assert oracle.validate([3, -2, 4]) == oracle.INVALID
    assert oracle.validate([3, 4]) == oracle.OK
    big = 1 << 21                                            # big^3 = 2^63
    assert oracle.validate([big, big, big]) == oracle.OVERFLOW
    assert oracle.validate([big - 1] * 3) == oracle.OK      # (2^21-1)^3 < 2^63
    assert oracle.validate([big - 1] * 4) == oracle.OVERFLOW  # 2 * (2^21-1)^3 > 2^63
    with pytest.raises(ValueError):
        oracle.fill([7])
    with pytest.raises(OverflowError):
        oracle.fill([big] * 3)


def test_large_values_exact():
    # Near the int64 limit: n = 3, dims 2^20, cost 2 * 2^60 = 2^61.
    p = [1 << 20] * 4
    m, s = oracle.fill(p)
    assert m[0, 2] == 2 * (1 << 60)
    assert s[0, 2] == 0


def test_check_cells_flags_planted_mistakes():
    p = workloads.uniform_dims(60, 1, 1024, 41)
    m, s = oracle.fill(p)
    cells = [(i, j) for i in range(60) for j in range(i + 1, 60)]
    assert oracle.check_cells(p, m, s, cells) == 0
    m2 = m.copy()
    m2[5, 30] += 1
    assert oracle.check_cells(p, m2, s, [(5, 30)]) == 1
    s2 = s.copy()
    s2[3, 40] = s2[3, 40] + 1 if s2[3, 40] + 1 < 40 else s2[3, 40] - 1
    assert oracle.check_cells(p, m, s2, [(3, 40)]) == 1
    assert oracle.check_cells(p, m, s, [(4, 4)]) == 1   # not an i < j cell
