"""Optimal order read back on the GPU (mcm_parenthesize*) vs the oracle.

Node intervals and costs are integers: compared exactly.  Tables come from
the oracle's fill or from the synthetic split-table shapes (never from the
GPU solve, except in the end-to-end cases, which check against properties
and the oracle's own tables).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import paren
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


def _device_table(s):
    import torch
    return torch.from_numpy(np.ascontiguousarray(s, dtype=np.int32)).cuda()


def _check(p, s, tag):
    """GPU read-back of table s equals the oracle's, bit for bit."""
    import torch
    n = s.shape[0]
    _say(f"[gpu] parenthesize {tag} n={n}")
    lo, hi, cost, text = binding.parenthesize(_device_table(s), p=p)
    torch.cuda.synchronize()
    olo, ohi, ocost, otext = paren.reconstruct(p, s)
    assert np.array_equal(lo.cpu().numpy(), olo), f"{tag}: lo differs"
    assert np.array_equal(hi.cpu().numpy(), ohi), f"{tag}: hi differs"
    assert cost == ocost, f"{tag}: cost {cost} vs {ocost}"
    assert text == otext, f"{tag}: text differs"
    return cost


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 130, 333, 700])
def test_optimal_tables(n):
    p = workloads.uniform_dims(n, 1, 1024, 500 + n)
    m, s = oracle.fill(p, threads=oracle.default_threads())
    cost = _check(p, s, "uniform")
    assert cost == m[0][n - 1]


@pytest.mark.parametrize("kind", ["equal", "increasing", "decreasing", "alternating", "ties"])
def test_structured_dims(kind):
    n = 257
    p = {"equal": workloads.all_equal(n, 9), "increasing": workloads.increasing(n),
         "decreasing": workloads.decreasing(n), "alternating": workloads.alternating(n),
         "ties": workloads.tie_heavy(n, 7)}[kind]
    m, s = oracle.fill(p, threads=oracle.default_threads())
    assert _check(p, s, kind) == m[0][n - 1]


@pytest.mark.parametrize("shape", workloads.SPLIT_SHAPES)
@pytest.mark.parametrize("n", [2, 66, 2049, 4500])
def test_tree_shapes(shape, n):
    # Long spines cross the 2048-entry LDS window and many register
    # sub-windows; zigzag changes direction at every node.
    if shape == "zigzag" and n > 2100:
        n = 2100
    p = workloads.uniform_dims(n, 1, 1024, 7)
    _check(p, workloads.split_table(n, shape, seed=n), shape)


def test_without_cost_or_intervals():
    import torch
    n = 300
    s = workloads.split_table(n, "random", seed=3)
    text = torch.empty(binding.parens_length(n) + 1, dtype=torch.uint8, device="cuda")
    binding.parenthesize_into(_device_table(s), n, text=text)
    torch.cuda.synchronize()
    raw = text.cpu().numpy().tobytes()
    assert raw[:-1].decode("ascii") == paren.parens_text(s, n) and raw[-1] == 0


def test_not_a_split_table():
    import torch
    n = 40
    p = workloads.uniform_dims(n, 1, 50, 1)
    s = workloads.split_table(n, "right", 0)
    s[0][n - 1] = n - 1
    _check(p, s, "bad root")
    s = workloads.split_table(n, "random", 5)
    # a cell on the tree's path, below the root
    lo, hi, ok = paren.tree_from_splits(s, n)
    k = next(k for k in range(n - 1) if hi[k] - lo[k] >= 3 and (lo[k], hi[k]) != (0, n - 1))
    s[lo[k]][hi[k]] = hi[k] + 5
    assert _check(p, s, "bad inner") == -1
    # entries above, at and below the cell's split range, on L and R walks
    for seed in range(9):
        s = workloads.split_table(n, "random", 40 + seed)
        lo, hi, ok = paren.tree_from_splits(s, n)
        ks = [k for k in range(n - 1) if hi[k] - lo[k] >= 2]
        k = ks[(7 * seed) % len(ks)]
        s[lo[k]][hi[k]] = [hi[k] + 5, lo[k] - 1, hi[k]][seed % 3]
        assert _check(p, s, f"bad {seed}") == -1
    torch.cuda.synchronize()


def test_batched_oracle_tables():
    import torch
    rng = np.random.default_rng(21)
    ns = np.array([1, 2, 3] + [int(v) for v in rng.integers(4, 400, size=60)] + [1, 700],
                  dtype=np.int32)
    dims = [workloads.uniform_dims(int(n), 1, 1024, 900 + b) for b, n in enumerate(ns)]
    tabs = [oracle.fill(p, threads=oracle.default_threads()) for p in dims]
    tab_off = binding.table_offsets(ns)
    node_off = binding.node_offsets(ns)
    s_all = np.concatenate([t[1].ravel() for t in tabs])
    p_all = np.concatenate(dims)
    p_off = np.concatenate([[0], np.cumsum([len(p) for p in dims])[:-1]]).astype(np.int64)
    g = max(int(node_off[-1] + ns[-1] - 1), 1)
    lo = torch.full((g,), -7, dtype=torch.int32, device="cuda")
    hi = torch.full((g,), -7, dtype=torch.int32, device="cuda")
    cost = torch.full((ns.size,), -7, dtype=torch.int64, device="cuda")
    _say(f"[gpu] parenthesize_batched count={ns.size}")
    binding.parenthesize_batched_into(ns, tab_off, _device_table(s_all), node_off, lo, hi,
                                      p_off=p_off, p_all=p_all, cost_all=cost)
    torch.cuda.synchronize()
    lo, hi, cost = lo.cpu().numpy(), hi.cpu().numpy(), cost.cpu().numpy()
    for b, n in enumerate(ns):
        n = int(n)
        olo, ohi, ocost, _ = paren.reconstruct(dims[b], tabs[b][1])
        o = int(node_off[b])
        assert np.array_equal(lo[o:o + n - 1], olo), f"chain {b}: lo"
        assert np.array_equal(hi[o:o + n - 1], ohi), f"chain {b}: hi"
        assert cost[b] == ocost == tabs[b][0][0][n - 1], f"chain {b}: cost"


def test_batched_workload_end_to_end():
    # The 4096-chain workload solved in one batched call, then every tree
    # read back in one launch; sampled chains against the oracle's tables.
    import torch
    batch = workloads.batched_4096()
    ns = batch.ns
    tab_off = binding.table_offsets(ns)
    node_off = binding.node_offsets(ns)
    total = int(tab_off[-1] + int(ns[-1]) ** 2)
    m_all = torch.empty(total, dtype=torch.int64, device="cuda")
    s_all = torch.empty(total, dtype=torch.int32, device="cuda")
    g = int(node_off[-1] + ns[-1] - 1)
    lo = torch.empty(g, dtype=torch.int32, device="cuda")
    hi = torch.empty(g, dtype=torch.int32, device="cuda")
    cost = torch.empty(ns.size, dtype=torch.int64, device="cuda")
    _say("[gpu] batched 4096 solve + parenthesize")
    binding.solve_batched_into(ns, batch.p_off, batch.p_all, tab_off, m_all, s_all)
    binding.parenthesize_batched_into(ns, tab_off, s_all, node_off, lo, hi, p_off=batch.p_off,
                                      p_all=batch.p_all, cost_all=cost)
    torch.cuda.synchronize()
    lo, hi, cost = lo.cpu().numpy(), hi.cpu().numpy(), cost.cpu().numpy()
    m_root = m_all[torch.as_tensor(tab_off + ns.astype(np.int64) - 1, device="cuda")]
    assert np.array_equal(cost, m_root.cpu().numpy()), "tree cost != m[0][n-1]"
    thr = oracle.default_threads()
    for b in list(range(0, ns.size, 257)) + [ns.size - 1]:
        n = int(ns[b])
        p = batch.dims(b)
        _, os_ = oracle.fill(p, threads=thr)
        olo, ohi, ocost, _ = paren.reconstruct(p, os_)
        o = int(node_off[b])
        assert np.array_equal(lo[o:o + n - 1], olo) and np.array_equal(hi[o:o + n - 1], ohi)
        assert cost[b] == ocost


def test_benchmark_chain_full_size(n8192_oracle):
    # n = 8192, the benchmark chain: the tree the GPU reads back from the
    # GPU's own table equals the oracle's read-back of the oracle's table
    # (intervals, cost and text), and its cost equals the solved m[0][n-1].
    import torch
    p, om, os_ = n8192_oracle
    n = len(p) - 1
    _say(f"[gpu] solve + parenthesize n={n}")
    m, s = binding.solve(p, algo="tiled")
    lo, hi, cost, text = binding.parenthesize(s, p=p)
    torch.cuda.synchronize()
    lo, hi = lo.cpu().numpy(), hi.cpu().numpy()
    _say("[cpu] oracle read-back n=8192")
    olo, ohi, ocost, otext = paren.reconstruct(p, os_)
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    assert cost == ocost == int(om[0, n - 1]) == int(m[0, n - 1].item())
    assert text == otext
    assert len(text) == binding.parens_length(n)
