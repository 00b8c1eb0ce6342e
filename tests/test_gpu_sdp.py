"""S-DP solver (mcm_sdp_solve) vs the oracle: int32, compared exactly."""
import sys

import numpy as np
import pytest

from oracle import sdp
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


def _run(a, init, n, op):
    import torch
    st = torch.full((n,), 12345, dtype=torch.int32, device="cuda")
    st[:int(a[0])] = torch.from_numpy(np.asarray(init, dtype=np.int32)[:int(a[0])]).cuda()
    _say(f"[gpu] sdp n={n} k={len(a)} a1={int(a[0])} op={op}")
    binding.sdp_solve_into(a, st, op)
    torch.cuda.synchronize()
    return st.cpu().numpy()


@pytest.mark.parametrize("op", sdp.OPS)
@pytest.mark.parametrize("seed", range(6))
def test_random_small(op, seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 300))
    top = int(rng.integers(k, 4 * k + 20))
    a = np.sort(rng.choice(top, size=k, replace=False) + 1)[::-1].astype(np.int32)
    n = int(a[0] + rng.integers(0, 9000))
    init = rng.integers(-(1 << 30), 1 << 30, size=int(a[0])).astype(np.int32)
    assert np.array_equal(_run(a, init, n, op), sdp.solve(a, init, n, op))


@pytest.mark.parametrize("case", ["fib", "one", "consecutive", "sparse", "edge"])
def test_structured(case):
    if case == "fib":
        a, init, n, op = np.array([2, 1]), np.array([1, 1]), 5000, "add"
    elif case == "one":
        a, init, n, op = np.array([7]), np.arange(7) * 3 - 9, 4100, "min"
    elif case == "consecutive":
        a, init = workloads.sdp_instance(0, 200, 0, "consecutive")
        n, op = 6000, "min"
    elif case == "sparse":
        # offsets far apart: many small far chunks
        a = np.array([9000, 7001, 5003, 2048, 2047, 64, 63, 1])
        init, n, op = np.random.default_rng(4).integers(0, 1000, size=9000), 16000, "max"
    else:
        # a_1 = n (nothing to compute) and a_1 = n - 1
        a, init, op = np.array([50, 3]), np.arange(50), "min"
        assert np.array_equal(_run(a, init, 50, op), sdp.solve(a, init, 50, op))
        n = 51
    assert np.array_equal(_run(a, init, n, op), sdp.solve(a, init, n, op))


def test_table1_small_config():
    n, k = workloads.SDP_CONFIGS["sdp_small"]
    a, init = workloads.sdp_instance(n, k, 11)
    assert np.array_equal(_run(a, init, n, "min"), sdp.solve(a, init, n, "min"))


def _sampled_recurrence(st, a, init, op, count, seed):
    assert np.array_equal(st[:int(a[0])], init)
    rng = np.random.default_rng(seed)
    n = st.size
    idx = np.unique(np.concatenate([rng.integers(int(a[0]), n, size=count),
                                    [int(a[0]), n - 1]]))
    a64 = a.astype(np.int64)
    for c in range(0, idx.size, 128):
        ii = idx[c:c + 128]
        vals = st[ii[:, None] - a64[None, :]]
        if op == "min":
            want = vals.min(axis=1)
        elif op == "max":
            want = vals.max(axis=1)
        else:
            want = (vals.astype(np.uint32).sum(axis=1, dtype=np.uint64) & 0xFFFFFFFF)
            want = want.astype(np.uint32).view(np.int32)
        assert np.array_equal(st[ii], want)


def test_table1_medium_config_full():
    # Table I's middle range at its top (n = 2^17, k = 2^15): the whole table
    # against the oracle (a few seconds of numpy gathers per operator).
    n, k = workloads.SDP_CONFIGS["sdp_medium"]
    a, init = workloads.sdp_instance(n, k, 12)
    for op in ("min", "add"):
        _say(f"[gpu] sdp medium n={n} k={k} op={op}, full oracle")
        assert np.array_equal(_run(a, init, n, op), sdp.solve(a, init, n, op))


def test_table1_large_config_prefix_and_sampled():
    # The largest range (n = 2^19, k = 2^17): the oracle over the first 2^14
    # computed elements (every element depends only on earlier ones, so a
    # prefix of the table is the oracle's table of that length), and every
    # sampled element beyond it equal to the fold of its sources.
    n, k = workloads.SDP_CONFIGS["sdp_large"]
    a, init = workloads.sdp_instance(n, k, 12)
    cut = int(a[0]) + (1 << 14)
    for op in ("min", "add"):
        _say(f"[gpu] sdp large n={n} k={k} op={op}, oracle prefix {cut}")
        st = _run(a, init, n, op)
        assert np.array_equal(st[:cut], sdp.solve(a, init, cut, op))
        _sampled_recurrence(st, a, init, op, 1500, 3)


@pytest.mark.parametrize("op", sdp.OPS)
def test_old_and_new_offsets_full(op):
    # Offsets on both sides of two blocks (4096), several blocks and a ragged
    # last one: the far terms split between the two streams.
    rng = np.random.default_rng(21)
    a = np.sort(rng.choice(12000, size=3000, replace=False) + 1)[::-1].astype(np.int32)
    n = int(a[0]) + 5 * 2048 + 777
    init = rng.integers(-(1 << 30), 1 << 30, size=int(a[0])).astype(np.int32)
    assert (a >= 4096).any() and (a < 4096).any()
    assert np.array_equal(_run(a, init, n, op), sdp.solve(a, init, n, op))


def test_consecutive_beyond_two_blocks():
    # Fig. 4's worst case with k above 2B: offsets k..1 fall on both sides.
    a, init = workloads.sdp_instance(0, 6000, 2, "consecutive")
    n = 6000 + 4 * 2048 + 5
    assert np.array_equal(_run(a, init, n, "min"), sdp.solve(a, init, n, "min"))
