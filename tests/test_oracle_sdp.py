"""Pins for the S-DP oracle (no GPU).

The S-DP oracle is Eq. (1) in the loop order of Fig. 1.  It is pinned to
the paper's own Fibonacci example, closed forms (one offset, consecutive
offsets), an independent reachability / path-counting definition on small
inputs, and the lockstep run of the pipeline of Fig. 2 (with its step
count).
"""
import random

import numpy as np
import pytest

from oracle import sdp


def test_fibonacci_example():
    # Section II-A: k = 2, a = (2, 1), addition, ST[0] = ST[1] = 1 gives the
    # Fibonacci numbers.
    n = 60
    st = sdp.solve([2, 1], [1, 1], n, "add")
    fib = [1, 1]
    while len(fib) < n:
        fib.append(fib[-1] + fib[-2])
    assert [int(v) & 0xFFFFFFFF for v in st] == [f % (1 << 32) for f in fib]
    assert list(st[:8]) == [1, 1, 2, 3, 5, 8, 13, 21]


@pytest.mark.parametrize("op", sdp.OPS)
def test_single_offset_is_periodic(op):
    rng = np.random.default_rng(1)
    d, n = 7, 100
    init = rng.integers(-1000, 1000, size=d).astype(np.int32)
    st = sdp.solve([d], init, n, op)
    assert np.array_equal(st, init[np.arange(n) % d])


def test_consecutive_offsets_closed_form():
    # The worst case of Fig. 4 (a = k, k-1, ..., 1): from ST[k] on every
    # element is the minimum (maximum) of the preset values.
    k, n = 9, 80
    init = np.random.default_rng(2).integers(-50, 50, size=k).astype(np.int32)
    a = list(range(k, 0, -1))
    assert np.all(sdp.solve(a, init, n, "min")[k:] == init.min())
    assert np.all(sdp.solve(a, init, n, "max")[k:] == init.max())


def _reachable_preset(a, i, a1, memo):
    """Preset indices reachable from i by subtracting offsets, every
    intermediate index being a computed one (>= a_1)."""
    if i < a1:
        return {i}
    if i in memo:
        return memo[i]
    out = set()
    for d in a:
        out |= _reachable_preset(a, i - d, a1, memo)
    memo[i] = out
    return out


def _paths(a, i, a1, memo):
    """Number of offset sequences from i to each preset index (a dict)."""
    if i < a1:
        return {i: 1}
    if i in memo:
        return memo[i]
    out = {}
    for d in a:
        for x, c in _paths(a, i - d, a1, memo).items():
            out[x] = out.get(x, 0) + c
    memo[i] = out
    return out


@pytest.mark.parametrize("seed", range(25))
def test_against_reachability_and_path_counts(seed):
    rng = random.Random(seed)
    k = rng.randint(1, 5)
    a = sorted(rng.sample(range(1, 9), k), reverse=True)
    n = rng.randint(a[0], 40)
    init = [rng.randint(-100, 100) for _ in range(a[0])]
    mn = sdp.solve(a, init, n, "min")
    mx = sdp.solve(a, init, n, "max")
    ad = sdp.solve(a, init, n, "add")
    memo, pm = {}, {}
    for i in range(n):
        reach = _reachable_preset(a, i, a[0], memo)
        assert mn[i] == min(init[x] for x in reach)
        assert mx[i] == max(init[x] for x in reach)
        total = sum(c * init[x] for x, c in _paths(a, i, a[0], pm).items())
        assert int(ad[i]) & 0xFFFFFFFF == total % (1 << 32)


@pytest.mark.parametrize("seed", range(30))
def test_fig2_pipeline_matches_definition(seed):
    rng = random.Random(1000 + seed)
    k = rng.randint(1, 8)
    a = sorted(rng.sample(range(1, 16), k), reverse=True)
    n = rng.randint(a[0], 60)
    init = [rng.randint(-1000, 1000) for _ in range(a[0])]
    for op in sdp.OPS:
        st, steps = sdp.pipeline(a, init, n, op)
        assert np.array_equal(st, sdp.solve(a, init, n, op))
        # the outer loop of Fig. 2 runs from a_1 to n + k - 2
        assert steps == max(n + k - 1 - a[0], 0)


def test_validation():
    with pytest.raises(ValueError):
        sdp.solve([], [], 5)
    with pytest.raises(ValueError):
        sdp.solve([2, 2], [0, 0], 5)          # not strictly decreasing
    with pytest.raises(ValueError):
        sdp.solve([3, 0], [0, 0, 0], 5)       # a_k must be positive
    with pytest.raises(ValueError):
        sdp.solve([6], [0] * 6, 5)            # a_1 > n
    st = sdp.solve([5], [1, 2, 3, 4, 5], 5)   # a_1 = n: nothing to compute
    assert list(st) == [1, 2, 3, 4, 5]
