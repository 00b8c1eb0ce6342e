"""The C ABI library on the CPU: it loads, exports every declared symbol,
and rejects bad input before any device call (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2008_01938_amd import binding, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.lib_path()):
        pytest.skip("libmcm.so not built")
    return binding.load()


def test_header_declares_expected_functions():
    assert _declared_functions() == sorted(binding.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for st in range(6):
        assert binding.status_string(st)
    assert binding.status_string(99) == "unknown status"
    assert binding.version() >= 100


def test_check_chain(lib):
    assert binding.check_chain([3, 4]) == binding.OK
    assert binding.check_chain([3]) == binding.ERR_INVALID_ARG          # n = 0
    assert binding.check_chain([3, 0, 4]) == binding.ERR_INVALID_ARG
    assert binding.check_chain([3, -1, 4]) == binding.ERR_INVALID_ARG
    big = 1 << 21
    assert binding.check_chain([big] * 3) == binding.ERR_OVERFLOW
    assert binding.check_chain([big - 1] * 3) == binding.OK
    assert lib.mcm_check_chain(None, 4) == binding.ERR_INVALID_ARG


def test_select_algo(lib):
    assert binding.select_algo(workloads.single_n8192()) == binding.ALGO_TILED
    assert binding.select_algo(workloads.single_n128()) == binding.ALGO_TILED
    # (n-1) * pmax^3 >= 2^46 leaves too few fp64 bits: the int64 tiled kernels.
    assert binding.select_algo([1 << 16] * 5) == binding.ALGO_TILED
    assert binding.select_algo([0, 1]) == -binding.ERR_INVALID_ARG
    assert binding.select_algo([1 << 21] * 3) == -binding.ERR_OVERFLOW


def _solve_raw(lib, p, m_ptr, s_ptr, algo=0):
    a = np.ascontiguousarray(np.asarray(p, dtype=np.int32))
    return lib.mcm_solve_algo(a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), a.size - 1,
                              ctypes.c_void_p(m_ptr), ctypes.c_void_p(s_ptr), algo,
                              ctypes.c_void_p(0))


def test_solve_rejects_bad_input_before_device(lib):
    # Host buffers stand in for device pointers: validation must fail before
    # anything is enqueued, so they are never touched.
    m = np.full(16, 7, dtype=np.int64)
    s = np.full(16, 7, dtype=np.int32)
    mp, sp = m.ctypes.data, s.ctypes.data
    assert _solve_raw(lib, [3], mp, sp) == binding.ERR_INVALID_ARG
    assert _solve_raw(lib, [3, 0, 2], mp, sp) == binding.ERR_INVALID_ARG
    assert _solve_raw(lib, [1 << 21] * 3, mp, sp) == binding.ERR_OVERFLOW
    assert _solve_raw(lib, [2, 3, 4], 0, sp) == binding.ERR_INVALID_ARG
    assert _solve_raw(lib, [2, 3, 4], mp, 0) == binding.ERR_INVALID_ARG
    assert _solve_raw(lib, [2, 3, 4], mp + 4, sp) == binding.ERR_INVALID_ARG   # misaligned
    assert _solve_raw(lib, [2, 3, 4], mp, sp + 2) == binding.ERR_INVALID_ARG
    assert _solve_raw(lib, [2, 3, 4], mp, sp, algo=9) == binding.ERR_INVALID_ARG
    assert _solve_raw(lib, [2] * 1100, mp, sp, algo=binding.ALGO_PIPELINE) == \
        binding.ERR_UNSUPPORTED                                                # n > 1025
    assert np.all(m == 7) and np.all(s == 7)


def test_noalloc_rejects_bad_input_before_device(lib):
    # As mcm_solve, plus the size limit of the fixed array; host buffers
    # stand in for device pointers and are never touched.
    m = np.full(16, 7, dtype=np.int64)
    s = np.full(16, 7, dtype=np.int32)
    mp, sp = ctypes.c_void_p(m.ctypes.data), ctypes.c_void_p(s.ctypes.data)

    def call(p, mp=mp, sp=sp):
        a = np.ascontiguousarray(np.asarray(p, dtype=np.int32))
        return lib.mcm_solve_noalloc(a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     a.size - 1, mp, sp, ctypes.c_void_p(0))

    assert call([3]) == binding.ERR_INVALID_ARG
    assert call([3, 0, 2]) == binding.ERR_INVALID_ARG
    assert call([1 << 21] * 3) == binding.ERR_OVERFLOW
    assert call([2, 3, 4], mp=ctypes.c_void_p(0)) == binding.ERR_INVALID_ARG
    assert call([2, 3, 4], sp=ctypes.c_void_p(s.ctypes.data + 2)) == binding.ERR_INVALID_ARG
    assert call(np.ones(binding.NOALLOC_MAX_N + 2, dtype=np.int32)) == binding.ERR_UNSUPPORTED
    assert lib.mcm_solve_noalloc(None, 4, mp, sp, ctypes.c_void_p(0)) == binding.ERR_INVALID_ARG
    assert np.all(m == 7) and np.all(s == 7)


def test_noalloc_constants_match_header():
    text = open(HEADER).read()
    assert re.search(r"#define MCM_NOALLOC_MAX_N (\d+)", text).group(1) == \
        str(binding.NOALLOC_MAX_N)
    assert "#define MCM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)" in text
    assert binding.NOALLOC_SCRATCH_BYTES == 64 << 20


def test_profile_read_rejects_bad_class(lib):
    d = ctypes.c_double()
    n = ctypes.c_int64()
    assert lib.mcm_profile_read(99, ctypes.byref(d), ctypes.byref(n), ctypes.byref(d)) == \
        binding.ERR_INVALID_ARG


def test_bench_refuses_multi_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_chain_create_rejects_bad_input(lib):
    h = ctypes.c_void_p()
    bad = np.array([3, 0, 4], dtype=np.int32)
    st = lib.mcm_chain_create(bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2,
                              ctypes.c_void_p(0), ctypes.byref(h))
    assert st == binding.ERR_INVALID_ARG and not h.value
    assert lib.mcm_chain_n(None) == 0
    lib.mcm_chain_destroy(None, ctypes.c_void_p(0))   # NULL is ignored
    m = np.zeros(4, dtype=np.int64)
    s = np.zeros(4, dtype=np.int32)
    assert lib.mcm_chain_solve(None, 0, ctypes.c_void_p(m.ctypes.data),
                               ctypes.c_void_p(s.ctypes.data), ctypes.c_void_p(0)) == \
        binding.ERR_INVALID_ARG


def test_batched_rejects_bad_input_before_device(lib):
    i32 = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.POINTER(ctypes.c_int64)
    m = np.full(64, 7, dtype=np.int64)
    s = np.full(64, 7, dtype=np.int32)

    def call(ns, p_off, p_all, tab, count=None):
        ns = np.asarray(ns, dtype=np.int32)
        p_off = np.asarray(p_off, dtype=np.int64)
        p_all = np.asarray(p_all, dtype=np.int32)
        tab = np.asarray(tab, dtype=np.int64)
        return lib.mcm_solve_batched(ns.size if count is None else count, ns.ctypes.data_as(i32),
                                     p_off.ctypes.data_as(i64), p_all.ctypes.data_as(i32),
                                     tab.ctypes.data_as(i64), ctypes.c_void_p(m.ctypes.data),
                                     ctypes.c_void_p(s.ctypes.data), ctypes.c_void_p(0))

    assert call([2, 0], [0, 0], [3, 4, 5], [0, 4]) == binding.ERR_INVALID_ARG      # n = 0
    assert call([2, 1], [0, 1], [3, 0, 5], [0, 4]) == binding.ERR_INVALID_ARG      # p = 0
    assert call([2], [-1], [3, 4, 5], [0]) == binding.ERR_INVALID_ARG              # offset
    assert call([2], [0], [1 << 21] * 3, [0]) == binding.ERR_OVERFLOW
    assert call([2], [0], [3, 4, 5], [0], count=-1) == binding.ERR_INVALID_ARG
    assert call([], [], [], [], count=0) == binding.OK                             # no-op
    # Tables that overlap would race between concurrent tiles: chain 1's
    # 2x2 table at offset 3 overlaps chain 0's [0, 4); in either order.
    assert call([2, 2], [0, 0], [3, 4, 5], [0, 3]) == binding.ERR_INVALID_ARG
    assert call([2, 2], [0, 0], [3, 4, 5], [3, 0]) == binding.ERR_INVALID_ARG
    assert call([3, 2, 1], [0, 0, 0], [3, 4, 5, 6], [20, 0, 3]) == binding.ERR_INVALID_ARG
    assert np.all(m == 7) and np.all(s == 7)


def test_plan_rejects_bad_input_before_device(lib):
    i32 = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.POINTER(ctypes.c_int64)

    def create(ns, p_off, tab, max_dim, count=None):
        ns = np.asarray(ns, dtype=np.int32)
        p_off = np.asarray(p_off, dtype=np.int64)
        tab = np.asarray(tab, dtype=np.int64)
        h = ctypes.c_void_p()
        st = lib.mcm_plan_create(ns.size if count is None else count, ns.ctypes.data_as(i32),
                                 p_off.ctypes.data_as(i64), tab.ctypes.data_as(i64), max_dim,
                                 ctypes.byref(h))
        assert not h.value
        return st

    assert create([2, 0], [0, 0], [0, 4], 8) == binding.ERR_INVALID_ARG       # n = 0
    assert create([2], [-1], [0], 8) == binding.ERR_INVALID_ARG               # offset
    assert create([2], [0], [-4], 8) == binding.ERR_INVALID_ARG               # table offset
    assert create([2], [0], [0], 0) == binding.ERR_INVALID_ARG                # max_dim
    assert create([2], [0], [0], 1 << 21) == binding.ERR_OVERFLOW             # 1 * (2^21)^3
    assert create([2], [0], [0], 8, count=-1) == binding.ERR_INVALID_ARG
    assert create([2, 2], [0, 0], [0, 2], 8) == binding.ERR_INVALID_ARG       # tables overlap
    p = np.array([3, 4, 5], dtype=np.int32)
    m = np.zeros(4, dtype=np.int64)
    s = np.zeros(4, dtype=np.int32)
    assert lib.mcm_plan_solve(None, p.ctypes.data_as(i32), ctypes.c_void_p(m.ctypes.data),
                              ctypes.c_void_p(s.ctypes.data), ctypes.c_void_p(0)) == \
        binding.ERR_INVALID_ARG
    lib.mcm_plan_destroy(None)   # NULL is ignored


def test_server_request_bytes(lib):
    assert binding.server_request_bytes([3, 0, 4]) == 0
    small = binding.server_request_bytes([3, 4, 5])
    big = binding.server_request_bytes(np.full(1001, 7, dtype=np.int32))
    # dims, m (8 B) and s (4 B) tables at least, 256-byte aligned
    assert small >= 2 * 2 * 12 and small % 256 == 0
    assert big >= 1000 * 1000 * 12 and big > small


def test_parens_length_matches_oracle(lib):
    from oracle import paren
    for n in (1, 2, 9, 10, 11, 99, 100, 101, 999, 1000, 8192, 100000):
        assert binding.parens_length(n) == paren.parens_length(n)
    assert binding.parens_length(0) == -1


def test_parenthesize_rejects_bad_input_before_device(lib):
    # Host buffers stand in for device pointers; every case fails validation
    # before anything is enqueued.
    s = np.full(16, 7, dtype=np.int32)
    lo = np.full(4, 7, dtype=np.int32)
    cost = np.full(1, 7, dtype=np.int64)
    p = np.array([3, 4, 5, 6, 7], dtype=np.int32)
    pp = p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    vp = ctypes.c_void_p
    f = lib.mcm_parenthesize
    assert f(pp, 0, vp(s.ctypes.data), None, None, None, None, None) == binding.ERR_INVALID_ARG
    assert f(pp, 4, None, None, None, None, None, None) == binding.ERR_INVALID_ARG
    # lo without hi
    assert f(pp, 4, vp(s.ctypes.data), vp(lo.ctypes.data), None, None, None,
             None) == binding.ERR_INVALID_ARG
    # a cost needs p
    assert f(None, 4, vp(s.ctypes.data), None, None, vp(cost.ctypes.data), None,
             None) == binding.ERR_INVALID_ARG
    bad = np.array([3, 0, 5, 6, 7], dtype=np.int32)
    assert f(bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 4, vp(s.ctypes.data), None,
             None, vp(cost.ctypes.data), None, None) == binding.ERR_INVALID_ARG
    assert (s == 7).all() and (lo == 7).all() and (cost == 7).all()
    g = lib.mcm_parenthesize_batched
    ns = np.array([4, 0], dtype=np.int32)
    off = np.zeros(2, dtype=np.int64)
    i64 = ctypes.POINTER(ctypes.c_int64)
    i32 = ctypes.POINTER(ctypes.c_int32)
    assert g(0, None, None, None, None, None, None, None, None, None, None) == binding.OK
    assert g(2, ns.ctypes.data_as(i32), None, None, off.ctypes.data_as(i64), vp(s.ctypes.data),
             off.ctypes.data_as(i64), vp(lo.ctypes.data), vp(lo.ctypes.data), None,
             None) == binding.ERR_INVALID_ARG
    # node ranges [0, 3) and [2, 5) overlap (the split tables do not)
    ns2 = np.array([4, 4], dtype=np.int32)
    toff = np.array([0, 16], dtype=np.int64)
    noff = np.array([0, 2], dtype=np.int64)
    s2 = np.full(32, 7, dtype=np.int32)
    lo2 = np.full(8, 7, dtype=np.int32)
    assert g(2, ns2.ctypes.data_as(i32), None, None, toff.ctypes.data_as(i64),
             vp(s2.ctypes.data), noff.ctypes.data_as(i64), vp(lo2.ctypes.data),
             vp(lo2.ctypes.data), None, None) == binding.ERR_INVALID_ARG
    assert (s2 == 7).all() and (lo2 == 7).all()


def test_sdp_rejects_bad_input_before_device(lib):
    st = np.full(64, 7, dtype=np.int32)
    vp = ctypes.c_void_p(st.ctypes.data)
    f = lib.mcm_sdp_solve

    def call(a, op=0, n=64):
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
        return f(arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), arr.size, op, vp, n, None)

    assert call([3, 3]) == binding.ERR_INVALID_ARG        # not strictly decreasing
    assert call([3, 0]) == binding.ERR_INVALID_ARG        # a_k < 1
    assert call([65]) == binding.ERR_INVALID_ARG          # a_1 > n
    assert call([4, 1], op=7) == binding.ERR_INVALID_ARG  # unknown operator
    assert call([4, 1], n=0) == binding.ERR_INVALID_ARG
    assert f(None, 2, 0, vp, 64, None) == binding.ERR_INVALID_ARG
    assert call([64]) == binding.OK                       # a_1 = n: nothing to do
    assert (st == 7).all()


def test_obst_rejects_bad_input_before_device(lib):
    e = np.full(16, 7, dtype=np.int64)
    r = np.full(16, 7, dtype=np.int32)
    ep, rp = ctypes.c_void_p(e.ctypes.data), ctypes.c_void_p(r.ctypes.data)
    i32 = ctypes.POINTER(ctypes.c_int32)

    def call(p, q, n):
        pa = np.ascontiguousarray(np.asarray(p, dtype=np.int32))
        qa = np.ascontiguousarray(np.asarray(q, dtype=np.int32))
        return lib.mcm_obst_solve(pa.ctypes.data_as(i32), qa.ctypes.data_as(i32), n, ep, rp, None)

    assert call([1, -1, 2], [1, 1, 1, 1], 3) == binding.ERR_INVALID_ARG
    assert call([1, 1, 2], [1, 1, -1, 1], 3) == binding.ERR_INVALID_ARG
    assert call([1], [1, 1], -1) == binding.ERR_INVALID_ARG
    assert lib.mcm_obst_solve(None, None, 0, ep, rp, None) == binding.ERR_INVALID_ARG
    big = (1 << 31) - 1
    n = 1 << 20
    assert call(np.full(n, big), np.full(n + 1, big), n) == binding.ERR_OVERFLOW
    assert (e == 7).all() and (r == 7).all()
