"""Batched solves (mcm_solve_batched) vs the CPU oracle, bit-exact."""
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


def run_batch(batch: workloads.Batch):
    import torch
    ns = batch.ns
    off = binding.table_offsets(ns)
    total = int(off[-1] + int(ns[-1]) ** 2) if ns.size else 1
    m_all = torch.full((max(total, 1),), -9, dtype=torch.int64, device="cuda")
    s_all = torch.full((max(total, 1),), -9, dtype=torch.int32, device="cuda")
    _say(f"[gpu] batched count={ns.size} max_n={int(ns.max()) if ns.size else 0}")
    binding.solve_batched_into(ns, batch.p_off, batch.p_all, off, m_all, s_all)
    torch.cuda.synchronize()
    return off, m_all.cpu().numpy(), s_all.cpu().numpy()


def check_against_oracle(batch, off, m_all, s_all, which=None):
    thr = oracle.default_threads()
    idx = range(batch.ns.size) if which is None else which
    for b in idx:
        n = int(batch.ns[b])
        o = int(off[b])
        om, os_ = oracle.fill(batch.dims(b), threads=thr)
        gm = m_all[o:o + n * n].reshape(n, n)
        gs = s_all[o:o + n * n].reshape(n, n)
        assert np.array_equal(gm, om), f"chain {b} (n={n}): m differs"
        assert np.array_equal(gs, os_), f"chain {b} (n={n}): s differs"


def test_mixed_sizes_and_paths():
    rng = np.random.default_rng(11)
    chains = []
    for t in range(40):
        n = int(rng.integers(1, 330))
        chains.append(workloads.uniform_dims(n, 1, 1024, 100 + t))
    # Outside the fp64 keys' range: the int64 tiled kernels inside the batch.
    chains.append(workloads.uniform_dims(20, (1 << 19) - 9, 1 << 19, 5))
    chains += [workloads.all_equal(130, 7), workloads.tie_heavy(200, 3), np.array([5, 6])]
    batch = workloads.make_batch(chains)
    off, m_all, s_all = run_batch(batch)
    check_against_oracle(batch, off, m_all, s_all)


def test_shared_dims_and_gapped_tables():
    import torch
    p = workloads.uniform_dims(300, 1, 1024, 9)
    # Three chains read overlapping windows of one dims array.
    ns = np.array([300, 150, 64], dtype=np.int32)
    p_off = np.array([0, 100, 236], dtype=np.int64)
    tab = np.array([0, 300 * 300 + 17, 300 * 300 + 17 + 150 * 150 + 5], dtype=np.int64)
    total = int(tab[-1] + 64 * 64)
    m_all = torch.full((total,), -9, dtype=torch.int64, device="cuda")
    s_all = torch.full((total,), -9, dtype=torch.int32, device="cuda")
    binding.solve_batched_into(ns, p_off, p, tab, m_all, s_all)
    torch.cuda.synchronize()
    m_h, s_h = m_all.cpu().numpy(), s_all.cpu().numpy()
    for b in range(3):
        n, o, po = int(ns[b]), int(tab[b]), int(p_off[b])
        om, os_ = oracle.fill(p[po:po + n + 1])
        assert np.array_equal(m_h[o:o + n * n].reshape(n, n), om)
        assert np.array_equal(s_h[o:o + n * n].reshape(n, n), os_)
    # Gaps between tables are untouched.
    assert np.all(m_h[300 * 300:300 * 300 + 17] == -9)
    assert np.all(s_h[300 * 300 + 17 + 150 * 150:tab[2]] == -9)


def test_empty_batch_is_noop():
    import torch
    m = torch.zeros(4, dtype=torch.int64, device="cuda")
    s = torch.zeros(4, dtype=torch.int32, device="cuda")
    binding.solve_batched_into([], [], [1], [], m, s)
    torch.cuda.synchronize()


def test_batched_4096_config():
    # The batched benchmark workload: 4096 chains, n in [16, 512], dims in
    # [1, 256], seed 3 -- every chain checked against the oracle.
    batch = workloads.batched_4096()
    off, m_all, s_all = run_batch(batch)
    check_against_oracle(batch, off, m_all, s_all)


def _plan_solve(plan, p_all, total, autotune=False):
    import torch
    m_all = torch.full((max(total, 1),), -9, dtype=torch.int64, device="cuda")
    s_all = torch.full((max(total, 1),), -9, dtype=torch.int32, device="cuda")
    choice = plan.autotune(p_all, m_all, s_all) if autotune else None
    plan.solve_into(p_all, m_all, s_all)
    torch.cuda.synchronize()
    return m_all.cpu().numpy(), s_all.cpu().numpy(), choice


def test_plan_reused_for_new_dims():
    # One plan, solved for two dims arrays of the same shape.
    rng = np.random.default_rng(12)
    ns = [int(rng.integers(1, 330)) for _ in range(30)] + [64, 65, 128, 1]
    first = workloads.make_batch([workloads.uniform_dims(n, 1, 1024, 200 + t)
                                  for t, n in enumerate(ns)])
    second = workloads.make_batch([workloads.uniform_dims(n, 1, 1024, 400 + t)
                                   for t, n in enumerate(ns)])
    assert np.array_equal(first.p_off, second.p_off)
    off = binding.table_offsets(first.ns)
    total = int(off[-1] + int(first.ns[-1]) ** 2)
    _say(f"[gpu] plan count={len(ns)} max_dim=1024")
    with binding.Plan(first.ns, first.p_off, off, 1024) as plan:
        for batch in (first, second):
            m_all, s_all, _ = _plan_solve(plan, batch.p_all, total)
            check_against_oracle(batch, off, m_all, s_all)


def test_plan_wavefront_chains():
    # A dims bound outside the fp64 keys' exact range sends every chain of
    # the plan to the int64 tiled kernels.
    chains = [workloads.uniform_dims(n, (1 << 19) - 9, 1 << 19, 30 + n) for n in (1, 2, 7, 20)]
    batch = workloads.make_batch(chains)
    off = binding.table_offsets(batch.ns)
    total = int(off[-1] + int(batch.ns[-1]) ** 2)
    _say("[gpu] plan int64 tiles max_dim=2^19")
    with binding.Plan(batch.ns, batch.p_off, off, 1 << 19) as plan:
        m_all, s_all, _ = _plan_solve(plan, batch.p_all, total)
    check_against_oracle(batch, off, m_all, s_all)


def test_plan_rejects_dims_above_bound():
    import torch
    batch = workloads.make_batch([workloads.uniform_dims(40, 1, 100, 3)])
    off = binding.table_offsets(batch.ns)
    m_all = torch.full((1600,), -9, dtype=torch.int64, device="cuda")
    s_all = torch.full((1600,), -9, dtype=torch.int32, device="cuda")
    with binding.Plan(batch.ns, batch.p_off, off, 50) as plan:
        with pytest.raises(binding.MCMError):
            plan.solve_into(batch.p_all, m_all, s_all)   # dims up to 100 > 50
    torch.cuda.synchronize()
    assert bool((m_all == -9).all()) and bool((s_all == -9).all())


def test_plan_autotuned_4096_config():
    # The batched benchmark workload through an autotuned plan: every chain
    # equal to mcm_solve_batched's tables, a sample checked against the oracle.
    batch = workloads.batched_4096()
    off, m_ref, s_ref = run_batch(batch)
    total = m_ref.size
    _say("[gpu] plan autotune count=4096")
    with binding.Plan(batch.ns, batch.p_off, off, 256) as plan:
        m_all, s_all, choice = _plan_solve(plan, batch.p_all, total, autotune=True)
    assert choice >= 0
    assert np.array_equal(m_all, m_ref) and np.array_equal(s_all, s_ref)
    sample = np.random.default_rng(0).choice(batch.ns.size, 128, replace=False)
    check_against_oracle(batch, off, m_all, s_all, which=sample)


def test_plan_empty_and_mixed_paths():
    import torch
    # An empty plan solves nothing.
    m = torch.zeros(4, dtype=torch.int64, device="cuda")
    s = torch.zeros(4, dtype=torch.int32, device="cuda")
    with binding.Plan([], [], [], 8) as plan:
        plan.solve_into(np.array([1], dtype=np.int32), m, s)
    torch.cuda.synchronize()
    assert int(m.abs().sum()) == 0 and int(s.abs().sum()) == 0
    # A dims bound of 2^15 keeps n = 1, 2 in the fp64 keys' range and sends
    # longer chains to the int64 tiled kernels: both kinds in one plan.
    chains = [workloads.uniform_dims(n, 1, 1 << 15, 60 + n) for n in (2, 5, 1, 40, 2, 130)]
    batch = workloads.make_batch(chains)
    off = binding.table_offsets(batch.ns)
    total = int(off[-1] + int(batch.ns[-1]) ** 2)
    _say("[gpu] plan mixed paths max_dim=2^15")
    with binding.Plan(batch.ns, batch.p_off, off, 1 << 15) as plan:
        m_all, s_all, _ = _plan_solve(plan, batch.p_all, total)
    check_against_oracle(batch, off, m_all, s_all)


# --------------------------------------------------------------------------
# 32-edge tiles (batches of small chains) and the plan's configurations.
# --------------------------------------------------------------------------

TILE32_SIZES = [1, 2, 3, 31, 32, 33, 63, 64, 65, 95, 96, 97, 100, 127, 128, 129, 200, 255, 256,
                257, 333, 511, 512, 513, 700, 1000, 1024]


def test_plan_tile32_ragged_sizes():
    # Sizes around multiples of 32 (one tile, ragged last tiles, several
    # tile-diagonals), tie-heavy and all-equal dims, on 32-edge tiles.
    chains = [workloads.uniform_dims(n, 1, 1024, 500 + n) for n in TILE32_SIZES]
    chains += [workloads.tie_heavy(150, 8), workloads.all_equal(97, 1024),
               workloads.alternating(130)]
    batch = workloads.make_batch(chains)
    off = binding.table_offsets(batch.ns)
    total = int(off[-1] + int(batch.ns[-1]) ** 2)
    _say(f"[gpu] plan tile 32, count={batch.ns.size}")
    with binding.Plan(batch.ns, batch.p_off, off, 1024) as plan:
        plan.set_config(32)
        assert plan.config()["tile_edge"] == 32
        m_all, s_all, _ = _plan_solve(plan, batch.p_all, total)
    check_against_oracle(batch, off, m_all, s_all)


def test_plan_tile32_4096_config_and_oneshot_from_cache():
    # The batched benchmark workload on 32-edge tiles equals the 64-edge
    # one-shot tables (checked against the oracle in full above), and a
    # sample equals the oracle.  The pinned configuration enters the tuning
    # cache, so a one-shot batched solve of the same bucket then runs on
    # 32-edge tiles too, with the same bytes.
    import torch
    batch = workloads.batched_4096()
    off, m_ref, s_ref = run_batch(batch)
    total = m_ref.size
    _say("[gpu] plan tile 32 count=4096")
    with binding.Plan(batch.ns, batch.p_off, off, 256) as plan:
        assert [c["tile_edge"] for c in plan.candidates()] == [64, 64, 64, 64, 32]
        plan.set_config(32)
        m_all, s_all, _ = _plan_solve(plan, batch.p_all, total)
    assert np.array_equal(m_all, m_ref) and np.array_equal(s_all, s_ref)
    sample = np.random.default_rng(1).choice(batch.ns.size, 96, replace=False)
    check_against_oracle(batch, off, m_all, s_all, which=sample)
    with binding.Plan(batch.ns, batch.p_off, off, 256) as plan:
        assert plan.config() == {"tile_edge": 32, "pair_min_blocks": plan.config()[
            "pair_min_blocks"], "source": "cache"}
    _, m_one, s_one = run_batch(batch)
    assert np.array_equal(m_one, m_ref) and np.array_equal(s_one, s_ref)
    torch.cuda.synchronize()


def test_plan_configurations_and_autotune_record():
    import torch
    small = workloads.make_batch([workloads.uniform_dims(n, 1, 512, 70 + n)
                                  for n in (40, 300, 600)])
    big = workloads.make_batch([workloads.uniform_dims(n, 1, 512, 80 + n) for n in (40, 1100)])
    for batch, edges in ((small, [64, 64, 64, 64, 32]), (big, [64, 64, 64, 64])):
        off = binding.table_offsets(batch.ns)
        total = int(off[-1] + int(batch.ns[-1]) ** 2)
        with binding.Plan(batch.ns, batch.p_off, off, 512) as plan:
            assert [c["tile_edge"] for c in plan.candidates()] == edges
            assert all(c["ms"] is None for c in plan.candidates())
            with pytest.raises(binding.MCMError) as e:
                plan.set_config(48)
            assert e.value.status == binding.ERR_INVALID_ARG
            if 32 not in edges:
                with pytest.raises(binding.MCMError) as e:
                    plan.set_config(32)
                assert e.value.status == binding.ERR_UNSUPPORTED
            _say(f"[gpu] autotune count={batch.ns.size} max_n={int(batch.ns.max())}")
            m_all, s_all, choice = _plan_solve(plan, batch.p_all, total, autotune=True)
            cands = plan.candidates()
            assert 0 <= choice < len(cands)
            assert all(c["ms"] is not None and c["ms"] > 0 for c in cands)
            assert cands[choice]["ms"] == min(c["ms"] for c in cands)
            cfg = plan.config()
            assert cfg["source"] == "tuned" and cfg["tile_edge"] == cands[choice]["tile_edge"]
        check_against_oracle(batch, off, m_all, s_all)
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
# Graph form of a plan: the whole solve recorded once, replayed per solve.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("edge", [64, 32, "int64"])
def test_plan_graph_replays_match_eager(edge):
    # Three replays with new dims each, the program's own eager solves and
    # synchronizations between them; every replay equals the eager plan
    # solve of the same dims (whole buffers) and the oracle.  "int64": a dims
    # bound beyond the fp64 keys' range puts every chain on the int64
    # schedule.
    import torch
    sizes = [1, 33, 64, 65, 150, 300, 513]
    max_dim = 1024 if edge != "int64" else 1 << 17

    def make(seed):
        return workloads.make_batch([workloads.uniform_dims(n, max_dim // 4, max_dim,
                                                            seed * 100 + n) for n in sizes])

    first = make(1)
    off = binding.table_offsets(first.ns)
    total = int(off[-1] + int(first.ns[-1]) ** 2)
    st = torch.cuda.Stream()
    m_g = torch.full((total,), -9, dtype=torch.int64, device="cuda")
    s_g = torch.full((total,), -9, dtype=torch.int32, device="cuda")
    with binding.Plan(first.ns, first.p_off, off, max_dim) as plan:
        if edge != "int64":
            plan.set_config(edge)
        _say(f"[gpu] plan graph capture, {edge}")
        plan.graph_create(m_g, s_g, stream=st)
        st.synchronize()
        for seed in (1, 2, 3):
            batch = make(seed)
            assert np.array_equal(batch.p_off, first.p_off)
            _say(f"[gpu] graph replay seed={seed}")
            plan.graph_solve(batch.p_all, stream=st)
            st.synchronize()
            m_e, s_e, _ = _plan_solve(plan, batch.p_all, total)   # eager, default stream
            torch.cuda.synchronize()
            assert np.array_equal(m_g.cpu().numpy(), m_e), f"replay {seed}: m"
            assert np.array_equal(s_g.cpu().numpy(), s_e), f"replay {seed}: s"
            check_against_oracle(batch, off, m_e, s_e)
