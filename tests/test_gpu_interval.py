"""Other interval DPs on the GPU: the optimal binary search tree
(mcm_obst_solve) against its oracle, exactly, and minimum-weight polygon
triangulation through the MCM entry point."""
import sys

import numpy as np
import pytest

from oracle import interval
from paper_2008_01938_amd import binding, workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()


def _solve(p, q, algo="auto"):
    import torch
    _say(f"[gpu] obst n={len(p)} algo={algo}")
    e, r = binding.obst_solve(p, q, algo=algo)
    torch.cuda.synchronize()
    return e.cpu().numpy(), r.cpu().numpy()


def test_textbook_example():
    e, r = _solve([15, 10, 5, 10, 20], [5, 10, 5, 5, 5, 10])
    assert e[0][5] == 275 and r[0][5] == 2


@pytest.mark.parametrize("algo", ["wavefront", "tiled"])
@pytest.mark.parametrize("n,hi,seed", [(1, 9, 1), (2, 1, 2), (7, 3, 3), (63, 7, 8), (64, 1000, 4),
                                       (65, 0, 5), (130, 50, 6), (160, 100000, 7), (200, 2, 9)])
def test_against_oracle(n, hi, seed, algo):
    rng = np.random.default_rng(seed)
    p = rng.integers(0, hi + 1, size=n).astype(np.int32)
    q = rng.integers(0, hi + 1, size=n + 1).astype(np.int32)
    e, r = _solve(p, q, algo)
    oe, orr = interval.obst_tables(p, q)
    assert np.array_equal(e, oe) and np.array_equal(r, orr)


def test_no_keys():
    e, r = _solve(np.zeros(0, dtype=np.int32), np.array([5], dtype=np.int32))
    assert e.tolist() == [[5]] and r.tolist() == [[-1]]


def test_tiled_range_and_fallback():
    # Weights too large for the fp64 keys: the tiled path refuses, AUTO
    # takes the int64 diagonal launches, and both agree with the oracle.
    n = 90
    rng = np.random.default_rng(12)
    p = rng.integers((1 << 31) - 1000, (1 << 31) - 1, size=n).astype(np.int32)
    q = rng.integers((1 << 31) - 1000, (1 << 31) - 1, size=n + 1).astype(np.int32)
    with pytest.raises(binding.MCMError):
        _solve(p, q, "tiled")
    e, r = _solve(p, q, "auto")
    oe, orr = interval.obst_tables(p, q)
    assert np.array_equal(e, oe) and np.array_equal(r, orr)


@pytest.mark.parametrize("algo", ["wavefront", "tiled"])
def test_n1200_whole_table_against_oracle(algo):
    # 1201 gaps (19 tiles of 64 per side, a ragged last one), weights below
    # 2^20: every cell and root against the oracle's by-length form.
    n = 1200
    rng = np.random.default_rng(10)
    p = rng.integers(0, 1 << 20, size=n).astype(np.int32)
    q = rng.integers(0, 1 << 20, size=n + 1).astype(np.int32)
    e, r = _solve(p, q, algo)
    oe, orr = _n1200_oracle(p, q)
    assert np.array_equal(e, oe) and np.array_equal(r, orr)


_ORACLE_CACHE = {}


def _n1200_oracle(p, q):
    key = (p.tobytes(), q.tobytes())
    if key not in _ORACLE_CACHE:
        _say("[cpu] optimal-BST oracle n=1200 (by interval length)")
        _ORACLE_CACHE[key] = interval.obst_tables_by_length(p, q)
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("algo", ["wavefront", "tiled"])
def test_large_sampled_recurrence(algo):
    # n = 3000: every sampled cell must satisfy the recurrence over the
    # table's own entries, with the smallest root; the diagonal holds q.
    n = 3000
    rng = np.random.default_rng(9)
    p = rng.integers(0, 1 << 20, size=n).astype(np.int64)
    q = rng.integers(0, 1 << 20, size=n + 1).astype(np.int64)
    e, r = _solve(p.astype(np.int32), q.astype(np.int32), algo)
    assert np.array_equal(np.diag(e), q) and np.array_equal(e, e.T)
    cq = np.concatenate([[0], np.cumsum(q)])
    cp = np.concatenate([[0], np.cumsum(p)])
    for _ in range(400):
        a = int(rng.integers(0, n))
        b = int(rng.integers(a + 1, n + 1))
        cand = e[a, a:b] + e[a + 1:b + 1, b] + (cq[b + 1] - cq[a]) + (cp[b] - cp[a])
        assert e[a, b] == cand.min()
        assert r[a, b] == a + 1 + int(np.argmin(cand))


def _triangulations(i, j):
    """Every triangulation of the convex polygon with vertices i..j, as
    lists of triangles (i < k < j)."""
    if j - i < 2:
        return [[]]
    out = []
    for k in range(i + 1, j):
        for left in _triangulations(i, k):
            for right in _triangulations(k, j):
                out.append(left + right + [(i, k, j)])
    return out


@pytest.mark.parametrize("seed", range(4))
def test_polygon_triangulation_is_mcm(seed):
    # A convex polygon with vertex weights v_0..v_m: the cheapest
    # triangulation, a triangle costing the product of its three vertex
    # weights, is the matrix chain of m matrices with p = v.
    import torch
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 9))
    v = rng.integers(1, 40, size=m + 1).astype(np.int32)
    best = min(sum(int(v[a]) * int(v[b]) * int(v[c]) for a, b, c in t)
               for t in _triangulations(0, m))
    mm, _ = binding.solve(v)
    torch.cuda.synchronize()
    assert int(mm[0, m - 1].item()) == best
