"""The int64 tiled kernels (chains whose costs pass the fp64 keys' exact
range, up to the int64 limit) vs the CPU oracle, bit-exact."""
import sys

import numpy as np
import pytest

import oracle
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


def pmax_for(n: int, bits: int = 63) -> int:
    """Largest dim with (n-1) * dim^3 < 2^bits."""
    d = int(round(((1 << bits) / max(n - 1, 1)) ** (1 / 3))) + 2
    while (n - 1) * d ** 3 >= (1 << bits):
        d -= 1
    return d


def check(p, algo="tiled"):
    import torch
    n = len(p) - 1
    _say(f"[gpu] wide solve n={n} pmax={int(np.max(p))} algo={algo}")
    m, s = binding.solve(p, algo=algo)
    torch.cuda.synchronize()
    om, os_ = oracle.fill(p, threads=oracle.default_threads())
    mh, sh = m.cpu().numpy(), s.cpu().numpy()
    for name, got, want in (("m", mh, om), ("s", sh, os_)):
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            i, j = bad[0]
            raise AssertionError(f"n={n}: {name} differs at {len(bad)} cells, first ({i},{j}): "
                                 f"gpu {got[i, j]} oracle {want[i, j]}")


SIZES = [1, 2, 3, 5, 63, 64, 65, 127, 129, 200, 300, 450]


@pytest.mark.parametrize("n", SIZES)
def test_near_int64_limit(n):
    # Every candidate cost can approach 2^63: dims in the top half of the
    # largest range the int64 bound allows.
    d = pmax_for(n)
    p = workloads.uniform_dims(n, d // 2, d, 6300 + n)
    assert binding.select_algo(p) == binding.ALGO_TILED
    check(p)


@pytest.mark.parametrize("n", [70, 257])
def test_wide_random_and_ties(n):
    d = pmax_for(n, 60)
    check(workloads.uniform_dims(n, 1, d, 6400 + n))                     # wide spread
    check(np.where(workloads.tie_heavy(n, 5) == 1, d - 1, d).astype(np.int32))  # many ties


def test_wide_all_equal_closed_form():
    import torch
    n = 300
    d = pmax_for(n)
    p = workloads.all_equal(n, d)
    _say(f"[gpu] wide all-equal n={n} d={d}")
    m, s = binding.solve(p, algo="tiled")
    torch.cuda.synchronize()
    iu, ju = np.triu_indices(n, 1)
    mh, sh = m.cpu().numpy(), s.cpu().numpy()
    assert np.array_equal(mh[iu, ju], (ju - iu).astype(np.int64) * d ** 3)
    assert np.array_equal(sh[iu, ju], iu.astype(np.int32))
    assert int(mh[0, n - 1]) == (n - 1) * d ** 3 and int(mh[0, n - 1]) < (1 << 63)


@pytest.mark.parametrize("top", [65535, 65536])
def test_wide_dims_at_the_32bit_product_bound(top):
    # Below 2^16 every product p_i p_k fits 32 bits and the kernels take the
    # 32 x 32-bit multiply; at 2^16 they take the 64 x 32-bit one.  Both
    # sides of the bound, dims in [top/2, top] and one dim equal to top.
    n = 300
    p = workloads.uniform_dims(n, top // 2, top, 6500 + top % 7)
    p[n // 3] = top
    assert (n - 1) * top ** 3 >= (1 << 46) and (n - 1) * top ** 3 < (1 << 63)
    assert binding.select_algo(p) == binding.ALGO_TILED
    check(p)


@pytest.mark.parametrize("over", [0, 1])
def test_wide_costs_at_the_2_53_bound(over):
    # (n-1) max(p)^3 just below 2^53: costs are exact fp64 integers and the
    # bulk runs in fp64, carrying the split beside the cost; one above: the
    # int64 bulk.  Dims in [d/2, d], one dim equal to d.
    n = 200
    d = pmax_for(n, 53) + over
    p = workloads.uniform_dims(n, d // 2, d, 6600 + over)
    p[n // 2] = d
    assert ((n - 1) * d ** 3 < (1 << 53)) == (over == 0)
    assert (n - 1) * d ** 3 >= (1 << 46)
    check(p)


@pytest.mark.parametrize("over", [0, 1])
def test_wide_costs_at_the_2_54_bound(over):
    # (n-1) max(p)^3 just below 2^54: the int64 closure carries keys
    # cost * 2^7 + local split; one above: (cost, split) pairs.
    n = 150
    d = pmax_for(n, 54) + over
    p = workloads.uniform_dims(n, d // 2, d, 6700 + over)
    p[n // 4] = d
    assert ((n - 1) * d ** 3 < (1 << 54)) == (over == 0)
    check(p)
    check(np.where(workloads.tie_heavy(n, 7 + over) == 1, d - 1, d).astype(np.int32))


def test_wide_matches_wavefront_path():
    import torch
    p = workloads.uniform_dims(333, 1, pmax_for(333), 77)
    m1, s1 = binding.solve(p, algo="tiled")
    m2, s2 = binding.solve(p, algo="wavefront")
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(s1, s2)


def test_n8192_dims_4096_whole_table():
    # n = 8192 with dims uniform in [1, 4096]: (n-1) * 4096^3 ~ 2^49, beyond
    # the fp64 keys; every cell against the oracle.
    p = workloads.uniform_dims(8192, 1, 4096, 4096)
    check(p)


def _mixed_batch(chains, mode, max_dim=None):
    import torch
    batch = workloads.make_batch(chains)
    off = binding.table_offsets(batch.ns)
    total = int(off[-1] + int(batch.ns[-1]) ** 2)
    m_all = torch.full((total,), -9, dtype=torch.int64, device="cuda")
    s_all = torch.full((total,), -9, dtype=torch.int32, device="cuda")
    _say(f"[gpu] mixed wide/fp64 batch, {mode}, ns={list(batch.ns)}")
    if mode == "oneshot":
        binding.solve_batched_into(batch.ns, batch.p_off, batch.p_all, off, m_all, s_all)
    else:
        with binding.Plan(batch.ns, batch.p_off, off, max_dim) as plan:
            plan.solve_into(batch.p_all, m_all, s_all)
    torch.cuda.synchronize()
    mh, sh = m_all.cpu().numpy(), s_all.cpu().numpy()
    for b in range(batch.ns.size):
        n, o = int(batch.ns[b]), int(off[b])
        om, os_ = oracle.fill(batch.dims(b))
        assert np.array_equal(mh[o:o + n * n].reshape(n, n), om), f"{mode} chain {b}"
        assert np.array_equal(sh[o:o + n * n].reshape(n, n), os_), f"{mode} chain {b}"


def test_batched_and_plan_mix_wide_and_fp64_chains():
    # One-shot: each chain's own dims decide its kernels.
    chains = [workloads.uniform_dims(n, 1, 1024, 900 + n) for n in (1, 40, 130, 300)]
    chains += [workloads.uniform_dims(n, pmax_for(n) // 2, pmax_for(n), 950 + n)
               for n in (2, 64, 150, 260)]
    _mixed_batch(chains, "oneshot")
    # Plan: one bound on the dims for every chain, 2^14, so chains with
    # (n-1) 2^42 < 2^46 (n <= 16) take the fp64 keys and the rest the int64
    # kernels.
    dmax = 1 << 14
    chains = [workloads.uniform_dims(n, 1, dmax, 960 + n) for n in (1, 5, 12, 16)]
    chains += [workloads.uniform_dims(n, dmax // 2, dmax, 970 + n)
               for n in (17, 64, 130, 260, 300)]
    _mixed_batch(chains, "plan", max_dim=dmax)
