"""GPU path vs the CPU oracle, bit-exact (integers: tolerance 0).

Every case prints its name, shape and kernel path before touching the GPU
so a failing run can be attributed.  Whole n x n buffers are compared
wherever the oracle can fill the table in seconds on the host's threads,
which includes the n = 8192 benchmark chain.  Beyond that (n = 16384, where
the bulk kernel stages with 64-bit offsets) the check uses oracle windows,
a large sample of cells re-evaluated from the table, and the closed form of
all-equal dimensions over the whole table.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2008_01938_amd import binding, workloads

pytestmark = pytest.mark.gpu

ALGOS = ["wavefront", "tiled"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_solve(p, algo="auto"):
    import torch
    _say(f"[gpu] solve n={len(p) - 1} algo={algo} pmax={int(np.max(p))}")
    m, s = binding.solve(p, algo=algo)
    torch.cuda.synchronize()
    return m.cpu().numpy(), s.cpu().numpy()


def assert_tables_equal(p, algo, threads=None):
    m, s = gpu_solve(p, algo)
    om, os_ = oracle.fill(p, threads=threads or oracle.default_threads())
    if not np.array_equal(m, om):
        bad = np.argwhere(m != om)
        i, j = bad[0]
        raise AssertionError(f"m differs at {len(bad)} cells, first ({i},{j}): "
                             f"gpu {m[i, j]} oracle {om[i, j]}")
    if not np.array_equal(s, os_):
        bad = np.argwhere(s != os_)
        i, j = bad[0]
        raise AssertionError(f"s differs at {len(bad)} cells, first ({i},{j}): "
                             f"gpu {s[i, j]} oracle {os_[i, j]}")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()


# Sizes around the tile edge (64) and its multiples: empty tile-diagonals,
# one tile, ragged last tile, several tile-diagonals with split chunks.
SIZES = [1, 2, 3, 4, 5, 7, 16, 33, 63, 64, 65, 100, 127, 128, 129, 191, 192, 193, 255, 257, 300,
         450]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n", SIZES)
def test_random_dims(algo, n):
    assert_tables_equal(workloads.uniform_dims(n, 1, 1024, 9000 + n), algo)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n", [6, 64, 130, 333])
def test_tie_heavy_dims(algo, n):
    assert_tables_equal(workloads.tie_heavy(n, 300 + n), algo)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("maker", ["all_equal", "increasing", "decreasing", "alternating"])
def test_structured_dims(algo, maker):
    n = 257
    p = {"all_equal": lambda: workloads.all_equal(n, 1024),
         "increasing": lambda: workloads.increasing(n),
         "decreasing": lambda: workloads.decreasing(n),
         "alternating": lambda: workloads.alternating(n)}[maker]()
    assert_tables_equal(p, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_config_n128(algo):
    assert_tables_equal(workloads.single_n128(), algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_config_n2048(algo):
    assert_tables_equal(workloads.single_n2048(), algo)


# Ragged mid sizes on the tiled path, whole tables: schedules in which the
# closure's wait for the interior sits in the end-block launch at every
# tile-diagonal (n up to about 4096) or only at the first and last ones,
# interiors chunked by their slack, last tiles 1 or 57 columns wide.
@pytest.mark.parametrize("n", [1025, 3001, 4097])
def test_ragged_mid_sizes_whole_table(n):
    assert_tables_equal(workloads.uniform_dims(n, 1, 1024, 9500 + n), "tiled")


def test_tie_heavy_n3001_whole_table():
    assert_tables_equal(workloads.tie_heavy(3001, 77), "tiled")


@pytest.mark.parametrize("algo", ["wavefront", "tiled", "auto"])
def test_large_values(algo):
    # Costs near 2^62: beyond the fp64 keys' exact range; the tiled path
    # runs its int64 kernels, the wavefront its int64 lanes.
    p = workloads.uniform_dims(32, (1 << 19) - 50, 1 << 19, 5)
    assert binding.select_algo(p) == binding.ALGO_TILED
    assert_tables_equal(p, algo)


def test_tiled_at_its_range_limit():
    # (n-1) * pmax^3 just under 2^46: the fewest fp64 bits the tiled path
    # accepts (7 bits of split index left).
    n = 300
    pmax = int(((1 << 46) // (n - 1)) ** (1 / 3)) - 1
    p = workloads.uniform_dims(n, pmax - 20, pmax, 8)
    assert binding.select_algo(p) == binding.ALGO_TILED
    assert_tables_equal(p, "tiled")


def test_profile_counts_every_split():
    import torch
    for algo, n in (("tiled", 300), ("wavefront", 150)):
        p = workloads.uniform_dims(n, 1, 1024, 77)
        binding.profile_enable(True)
        gpu_solve(p, algo)
        torch.cuda.synchronize()
        total = sum(binding.profile_read(c)["split_evals"] for c in range(5))
        binding.profile_enable(False)
        assert total == (n ** 3 - n) // 6, (algo, total)


def test_serial_profile_schedule_same_bytes():
    # The profiler's serial schedule (every launch on the caller's stream,
    # chunking fitted to the whole device) writes the same bytes and still
    # counts every split; switching it off restores the overlapped schedule.
    import torch
    p = workloads.uniform_dims(1500, 1, 1024, 1500)
    n = len(p) - 1
    binding.profile_enable(True, serial=True)
    try:
        m, s = gpu_solve(p, "tiled")
        torch.cuda.synchronize()
        total = sum(binding.profile_read(c)["split_evals"] for c in range(5))
        bulk = binding.profile_read(binding.PROF_BULK)
    finally:
        binding.profile_enable(False)
    assert total == (n ** 3 - n) // 6
    assert bulk["launches"] > 0 and bulk["ms"] > 0
    om, os_ = oracle.fill(p, threads=oracle.default_threads())
    assert np.array_equal(m, om) and np.array_equal(s, os_)
    m2, s2 = gpu_solve(p, "tiled")
    assert np.array_equal(m2, om) and np.array_equal(s2, os_)


def test_nondefault_stream_and_repeat_determinism():
    import torch
    p = workloads.uniform_dims(700, 1, 1024, 123)
    st = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(st):
            m, s = binding.solve(p, algo="tiled", stream=st)
        st.synchronize()
        outs.append((m.cpu().numpy(), s.cpu().numpy()))
    for m, s in outs[1:]:
        assert np.array_equal(m, outs[0][0]) and np.array_equal(s, outs[0][1])
    om, os_ = oracle.fill(p, threads=oracle.default_threads())
    assert np.array_equal(outs[0][0], om) and np.array_equal(outs[0][1], os_)


# --------------------------------------------------------------------------
# n = 8192, the benchmark configuration, in the launch configuration the
# benchmark times (algo auto -> tiled).
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def n8192():
    p = workloads.single_n8192()
    assert binding.select_algo(p) == binding.ALGO_TILED
    m, s = gpu_solve(p, "auto")
    return p, m, s


def test_n8192_whole_table_matches_oracle(n8192, n8192_oracle):
    # Every cell of both n x n buffers, against the oracle's own fill.
    p, m, s = n8192
    op, om, os_ = n8192_oracle
    assert np.array_equal(p, op)
    for name, got, want in (("m", m, om), ("s", s, os_)):
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            i, j = bad[0]
            raise AssertionError(f"{name} differs at {len(bad)} cells, first ({i},{j}): "
                                 f"gpu {got[i, j]} oracle {want[i, j]}")


def test_n8192_structure(n8192):
    p, m, s = n8192
    n = len(p) - 1
    pi = p.astype(np.int64)
    assert np.all(np.diag(m) == 0)
    assert np.array_equal(m, m.T)
    idx = np.arange(n - 1)
    assert np.array_equal(m[idx, idx + 1], pi[:-2] * pi[1:-1] * pi[2:])
    assert np.array_equal(s[idx, idx + 1], idx)
    il, jl = np.tril_indices(n)
    assert np.all(s[il, jl] == -1)
    iu, ju = np.triu_indices(n, 1)
    su = s[iu, ju]
    assert np.all((su >= iu) & (su < ju))


def test_n8192_windows_match_oracle(n8192):
    # Optimal substructure: the table of a sub-chain is a block of the
    # full table, so the oracle on windows checks every cell inside them.
    p, m, s = n8192
    rng = np.random.default_rng(8192)
    n = len(p) - 1
    for i0 in [0, n - 600] + list(rng.integers(0, n - 600, size=3)):
        i0 = int(i0)
        L = 600
        _say(f"[cpu] oracle window i0={i0} L={L}")
        wm, ws = oracle.fill(p[i0:i0 + L + 1], threads=oracle.default_threads())
        assert np.array_equal(m[i0:i0 + L, i0:i0 + L], wm)
        assert np.array_equal(s[i0:i0 + L, i0:i0 + L], np.where(ws >= 0, ws + i0, -1))


def test_n8192_sampled_recurrence(n8192):
    # The recurrence re-evaluated from the GPU table at sampled cells of
    # every size class, including the full-chain cell (0, n-1).
    p, m, s = n8192
    n = len(p) - 1
    rng = np.random.default_rng(1)
    i = rng.integers(0, n - 1, size=4000)
    d = np.minimum(rng.integers(1, n, size=4000), n - 1 - i)
    d = np.maximum(d, 1)
    cells = np.stack([i, i + d], axis=1)
    cells = np.concatenate([cells, [[0, n - 1], [1, n - 1], [0, n - 2]]])
    cells = cells[cells[:, 1] < n]
    assert oracle.check_cells(p, m, s, cells, threads=oracle.default_threads()) == 0


def test_n8192_all_equal_closed_form():
    n, d = 8192, 1024
    p = workloads.all_equal(n, d)
    m, s = gpu_solve(p, "auto")
    iu, ju = np.triu_indices(n, 1)
    assert np.array_equal(m[iu, ju], (ju - iu).astype(np.int64) * d ** 3)
    assert np.array_equal(s[iu, ju], iu.astype(np.int32))
    assert m[0, n - 1] == 8795019280384


def test_chain_api_matches_solve():
    import torch
    p = workloads.uniform_dims(333, 1, 1024, 4242)
    n = len(p) - 1
    _say("[gpu] chain api n=333")
    ch = binding.Chain(p)
    m = torch.empty((n, n), dtype=torch.int64, device="cuda")
    s = torch.empty((n, n), dtype=torch.int32, device="cuda")
    for algo in ("tiled", "wavefront", "auto"):
        m.fill_(-7)
        s.fill_(-7)
        ch.solve_into(m, s, algo=algo)
        torch.cuda.synchronize()
        om, os_ = oracle.fill(p, threads=oracle.default_threads())
        assert np.array_equal(m.cpu().numpy(), om) and np.array_equal(s.cpu().numpy(), os_)
    ch.close()
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
# n = 16384: the table passes 2 GiB, so the bulk kernel stages its panels
# with 64-bit offsets instead of 32-bit ones.
# --------------------------------------------------------------------------

def _device_closed_form(n, d):
    """Whole-table check of the all-equal closed form on the device:
    m[i][j] = |j - i| d^3 and s[i][j] = i above the diagonal, -1 elsewhere."""
    import torch
    p = workloads.all_equal(n, d)
    _say(f"[gpu] solve n={n} all dims {d} (closed form)")
    m, s = binding.solve(p, algo="auto")
    torch.cuda.synchronize()
    ar = torch.arange(n, device="cuda", dtype=torch.int64)
    for r0 in range(0, n, 2048):   # row blocks keep the expected tables small
        r = ar[r0:r0 + 2048, None]
        want_m = (ar[None, :] - r).abs() * (d ** 3)
        want_s = torch.where(ar[None, :] > r, r, torch.full_like(r, -1)).to(torch.int32)
        assert torch.equal(m[r0:r0 + 2048], want_m), f"m rows {r0}.."
        assert torch.equal(s[r0:r0 + 2048], want_s), f"s rows {r0}.."
    return m, s


def test_n16384_all_equal_closed_form():
    n, d = 16384, 1024
    assert binding.select_algo(workloads.all_equal(n, d)) == binding.ALGO_TILED
    m, s = _device_closed_form(n, d)
    assert int(m[0, n - 1].item()) == (n - 1) * d ** 3
    del m, s


def test_n16384_random_dims_windows_and_cells():
    # Random dims at n = 16384: oracle windows (optimal substructure makes
    # a window's table a block of the full one) at both ends and inside,
    # plus 10^6 cells spread over every distance class re-evaluated from
    # the table itself, including the full chain.
    import torch
    n = 16384
    p = workloads.uniform_dims(n, 1, 1024, 16384)
    assert binding.select_algo(p) == binding.ALGO_TILED
    _say(f"[gpu] solve n={n} random dims")
    mt, st = binding.solve(p, algo="auto")
    torch.cuda.synchronize()
    m, s = mt.cpu().numpy(), st.cpu().numpy()
    del mt, st
    thr = oracle.default_threads()
    rng = np.random.default_rng(16384)
    L = 700
    for i0 in [0, n - L] + [int(x) for x in rng.integers(0, n - L, size=3)]:
        _say(f"[cpu] oracle window i0={i0} L={L}")
        wm, ws = oracle.fill(p[i0:i0 + L + 1], threads=thr)
        assert np.array_equal(m[i0:i0 + L, i0:i0 + L], wm), f"window {i0}: m"
        assert np.array_equal(s[i0:i0 + L, i0:i0 + L], np.where(ws >= 0, ws + i0, -1)), \
            f"window {i0}: s"
    i = rng.integers(0, n - 1, size=1_000_000)
    d = np.maximum(np.minimum(rng.integers(1, n, size=i.size), n - 1 - i), 1)
    cells = np.stack([i, i + d], axis=1)
    cells = np.concatenate([cells, [[0, n - 1], [1, n - 1], [0, n - 2]]])
    _say(f"[cpu] recurrence at {len(cells)} cells")
    assert oracle.check_cells(p, m, s, cells, threads=thr) == 0
    assert np.all(np.diag(m) == 0)
    ar = np.arange(n)
    for r0 in range(0, n, 1024):   # row blocks: symmetry, and s = -1 on and below the diagonal
        rows = slice(r0, r0 + 1024)
        assert np.array_equal(m[rows], m[:, rows].T), f"m rows {r0}.. not symmetric"
        below = ar[None, :] <= ar[rows, None]
        assert np.all(s[rows][below] == -1), f"s rows {r0}.."
