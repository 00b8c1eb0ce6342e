"""The continuous-batching server: every served result equals the same
chain solved alone (and the oracle), under overlap, admission limits and
mixed kernel paths."""
import sys

import numpy as np
import pytest

import oracle
from paper_2008_01938_amd import binding, serve, workloads

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


# Arrival rate of the full-stream parity test: about 0.8 times the plain
# per-request capacity measured on one MI355X (about 850 requests/s).
SERVE_TEST_RATE = 700.0


def small_stream(count, rate, seed, n_hi=700):
    return workloads.serving_stream(count=count, rate=rate, seed=seed, n_lo=8, n_hi=n_hi)


def test_served_equals_alone_and_oracle():
    st = small_stream(80, rate=4000.0, seed=21)
    _say(f"[gpu] serve 80 requests, max n={int(st.batch.ns.max())}")
    res = serve.run_served(st, mem_budget=2 << 30, max_slots=64, keep=range(80))
    assert res.count == 80
    import torch
    for i in range(80):
        p = st.batch.dims(i)
        m_alone, s_alone = binding.solve(p)
        torch.cuda.synchronize()
        om, os_ = oracle.fill(p, threads=oracle.default_threads())
        m, s = res.outputs[i]
        assert np.array_equal(m, om) and np.array_equal(s, os_), f"request {i}"
        assert np.array_equal(m, m_alone.cpu().numpy()) and np.array_equal(s, s_alone.cpu().numpy())


def test_tiny_budget_forces_queueing():
    st = small_stream(30, rate=1e6, seed=5, n_hi=400)     # all arrive at once
    need = [binding.server_request_bytes(st.batch.dims(i)) for i in range(30)]
    budget = max(need) + 4096                             # about one request at a time
    _say(f"[gpu] serve with budget {budget} bytes")
    res = serve.run_served(st, mem_budget=budget, max_slots=64, keep=range(30))
    for i in range(30):
        om, os_ = oracle.fill(st.batch.dims(i))
        assert np.array_equal(res.outputs[i][0], om) and np.array_equal(res.outputs[i][1], os_)


def test_one_slot_serialises():
    st = small_stream(12, rate=1e6, seed=6, n_hi=300)
    res = serve.run_served(st, mem_budget=1 << 30, max_slots=1, keep=range(12))
    for i in range(12):
        om, os_ = oracle.fill(st.batch.dims(i))
        assert np.array_equal(res.outputs[i][0], om) and np.array_equal(res.outputs[i][1], os_)


def test_mixed_paths_and_errors():
    with binding.Server(1 << 30, 16) as srv:
        big = workloads.uniform_dims(30, (1 << 19) - 9, 1 << 19, 4)   # int64 wavefront
        small = workloads.uniform_dims(150, 1, 1024, 8)
        srv.submit(big, 1)
        srv.submit(small, 2)
        with pytest.raises(binding.MCMError) as e:
            srv.submit(np.array([3, 0, 4], dtype=np.int32), 3)
        assert e.value.status == binding.ERR_INVALID_ARG
        with pytest.raises(binding.MCMError) as e:
            srv.submit(workloads.uniform_dims(12000, 1, 4, 1), 4)      # > budget
        assert e.value.status == binding.ERR_NO_MEMORY
        got = {}
        t_end = binding.clock_now() + 60
        while len(got) < 2 and binding.clock_now() < t_end:
            for info in srv.poll():
                assert info.status == binding.OK
                got[int(info.tag)] = srv.fetch(info)
                srv.release(int(info.tag))
        assert set(got) == {1, 2}
        for tag, p in ((1, big), (2, small)):
            om, os_ = oracle.fill(p)
            assert np.array_equal(got[tag][0], om) and np.array_equal(got[tag][1], os_)
        with pytest.raises(binding.MCMError):
            srv.release(99)
        stats = srv.stats()
        assert stats["completed"] == 2 and stats["active"] == 0 and stats["bytes_in_use"] == 0


def test_few_large_requests_use_fine_chunks():
    # Two large requests alone on the server: each iteration cuts their
    # interiors into many chunks per tile (up to the cap), in proportion to
    # their work; results must still equal the oracle bit for bit.
    reqs = {7: workloads.uniform_dims(1800, 1, 1024, 31), 8: workloads.uniform_dims(2600, 1, 1024, 32)}
    _say("[gpu] serve two large requests (n=1800, n=2600)")
    got = {}
    with binding.Server(4 << 30, 4) as srv:
        for tag, p in reqs.items():
            srv.submit(p, tag)
        t_end = binding.clock_now() + 120
        while len(got) < 2 and binding.clock_now() < t_end:
            for info in srv.poll():
                assert info.status == binding.OK
                got[int(info.tag)] = srv.fetch(info)
                srv.release(int(info.tag))
    assert set(got) == set(reqs)
    for tag, p in reqs.items():
        om, os_ = oracle.fill(p, threads=oracle.default_threads())
        assert np.array_equal(got[tag][0], om) and np.array_equal(got[tag][1], os_), f"request {tag}"


def _d2d(dst, src_ptr: int, nbytes: int):
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    assert hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), nbytes,
                         3) == 0   # hipMemcpyDeviceToDevice


def test_benchmark_stream_served_equals_alone():
    # The benchmark's whole request stream (20000 requests, seed 4, n
    # log-uniform in [8, 4096], dims in [1, 1024]) at about 0.8 times the
    # plain per-request capacity: every served table equals the same chain
    # solved alone, compared on the device; every request with n <= 512 also
    # equals the oracle (on a pool of host threads, beside the serving loop).
    import concurrent.futures as cf

    import torch
    st = workloads.serving_stream(count=20000, rate=SERVE_TEST_RATE, seed=4)
    batch = st.batch
    count = int(batch.ns.size)
    _say(f"[gpu] serve benchmark stream, {count} requests, max n={int(batch.ns.max())}")
    done = 0
    futures = []

    def oracle_check(i, p, m_host, s_host):
        om, os_ = oracle.fill(p)
        return i, bool(np.array_equal(m_host, om) and np.array_equal(s_host, os_))

    pool = cf.ThreadPoolExecutor(max_workers=max(1, min(12, oracle.default_threads() - 2)))
    try:
        with binding.Server(24 << 30, 256) as srv:
            t0 = binding.clock_now()
            arrive = t0 + st.arrivals
            nxt = 0
            while done < count:
                now = binding.clock_now()
                while nxt < count and arrive[nxt] <= now:
                    srv.submit(batch.dims(nxt), nxt)
                    nxt += 1
                for info in srv.poll():
                    i, n = int(info.tag), int(info.n)
                    assert info.status == binding.OK, f"request {i}"
                    m_srv = torch.empty(n * n, dtype=torch.int64, device="cuda")
                    s_srv = torch.empty(n * n, dtype=torch.int32, device="cuda")
                    _d2d(m_srv, info.m, n * n * 8)
                    _d2d(s_srv, info.s, n * n * 4)
                    srv.release(i)
                    p = batch.dims(i)
                    m_alone, s_alone = binding.solve(p)
                    torch.cuda.synchronize()
                    assert torch.equal(m_srv.view(n, n), m_alone), f"request {i} (n={n}): m"
                    assert torch.equal(s_srv.view(n, n), s_alone), f"request {i} (n={n}): s"
                    if n <= 512:
                        futures.append(pool.submit(oracle_check, i, p,
                                                   m_srv.view(n, n).cpu().numpy(),
                                                   s_srv.view(n, n).cpu().numpy()))
                    done += 1
        for fu in futures:
            i, ok = fu.result()
            assert ok, f"request {i}: served table differs from the oracle"
    finally:
        pool.shutdown(wait=True)
    _say(f"[gpu] {done} served tables equal alone; {len(futures)} also equal the oracle")
    assert done == count and len(futures) == int(np.sum(batch.ns <= 512))


def test_duplicate_live_tag_is_rejected():
    # A tag names one request from submission to release; a second
    # submission under it is refused and the first completes normally.
    p = workloads.uniform_dims(100, 1, 1024, 55)
    with binding.Server(1 << 30, 8) as srv:
        srv.submit(p, 5)
        with pytest.raises(binding.MCMError) as e:
            srv.submit(p, 5)
        assert e.value.status == binding.ERR_INVALID_ARG
        got = []
        t_end = binding.clock_now() + 60
        while not got and binding.clock_now() < t_end:
            got = srv.poll()
        assert [int(x.tag) for x in got] == [5]
        with pytest.raises(binding.MCMError):   # polled, not released: still live
            srv.submit(p, 5)
        srv.release(5)
        srv.submit(p, 5)                        # free again after release
        got = []
        t_end = binding.clock_now() + 60
        while not got and binding.clock_now() < t_end:
            got = srv.poll()
        om, os_ = oracle.fill(p)
        m, s = srv.fetch(got[0])
        assert np.array_equal(m, om) and np.array_equal(s, os_)
        srv.release(5)
        stats = srv.stats()
        assert stats["completed"] == 2 and stats["active"] == 0 and stats["bytes_in_use"] == 0
