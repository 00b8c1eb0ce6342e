"""ctypes binding of ``libmcm.so`` (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; this module only
converts arguments.  PyTorch supplies device memory and the stream.  If the
library has not been built, every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

from .build import LIB

OK = 0
ERR_INVALID_ARG = 1
ERR_OVERFLOW = 2
ERR_NO_MEMORY = 3
ERR_DEVICE = 4
ERR_UNSUPPORTED = 5

ALGO_AUTO = 0
ALGO_WAVEFRONT = 1
ALGO_TILED = 2
ALGO_PIPELINE = 3
ALGOS = {"auto": ALGO_AUTO, "wavefront": ALGO_WAVEFRONT, "tiled": ALGO_TILED,
         "pipeline": ALGO_PIPELINE}

# Profiler kernel classes (mcm_profile_read).
PROF_SETUP, PROF_BULK, PROF_CLOSE, PROF_WAVE, PROF_BATCH = range(5)
PROFILE_SERIAL = 1 << 16   # MCM_PROFILE_SERIAL
PLAN_SOURCES = {0: "default", 1: "cache", 2: "tuned"}   # MCM_PLAN_*

# Every symbol include/mcm.h declares.
EXPORTED = (
    "mcm_status_string", "mcm_version", "mcm_check_chain", "mcm_select_algo",
    "mcm_solve", "mcm_solve_algo", "mcm_solve_noalloc", "mcm_solve_batched",
    "mcm_plan_create", "mcm_plan_solve", "mcm_plan_autotune", "mcm_plan_config",
    "mcm_plan_set_config", "mcm_plan_candidates", "mcm_plan_graph_create",
    "mcm_plan_graph_solve", "mcm_plan_destroy", "mcm_chain_create", "mcm_chain_solve",
    "mcm_chain_n", "mcm_chain_destroy", "mcm_server_create", "mcm_server_submit",
    "mcm_server_poll", "mcm_server_release", "mcm_server_request_bytes", "mcm_server_stats",
    "mcm_server_destroy", "mcm_clock_now", "mcm_profile_enable", "mcm_profile_enable_mask",
    "mcm_profile_read", "mcm_parens_length", "mcm_parenthesize", "mcm_parenthesize_batched",
    "mcm_sdp_solve", "mcm_obst_solve", "mcm_obst_solve_algo",
)
NOALLOC_MAX_N = 8192             # MCM_NOALLOC_MAX_N
NOALLOC_SCRATCH_BYTES = 64 << 20  # MCM_NOALLOC_SCRATCH_BYTES

SDP_OPS = {"min": 0, "max": 1, "add": 2}


class RequestInfo(ctypes.Structure):
    """mcm_request_info."""
    _fields_ = [("tag", ctypes.c_uint64), ("n", ctypes.c_int32), ("status", ctypes.c_int32),
                ("m", ctypes.c_void_p), ("s", ctypes.c_void_p), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class MCMError(RuntimeError):
    """A non-zero mcm_status from the library."""

    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return LIB


def load() -> ctypes.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB):
                raise RuntimeError(
                    f"{LIB} is not built; run `python -m paper_2008_01938_amd.build` "
                    "(or __graft_entry__.build())")
            lib = ctypes.CDLL(LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            vp = ctypes.c_void_p
            lib.mcm_status_string.argtypes = [ctypes.c_int32]
            lib.mcm_status_string.restype = ctypes.c_char_p
            lib.mcm_version.argtypes = []
            lib.mcm_version.restype = ctypes.c_int32
            lib.mcm_check_chain.argtypes = [i32p, ctypes.c_int32]
            lib.mcm_check_chain.restype = ctypes.c_int
            lib.mcm_select_algo.argtypes = [i32p, ctypes.c_int32]
            lib.mcm_select_algo.restype = ctypes.c_int32
            lib.mcm_solve.argtypes = [i32p, ctypes.c_int32, vp, vp, vp]
            lib.mcm_solve.restype = ctypes.c_int
            lib.mcm_solve_algo.argtypes = [i32p, ctypes.c_int32, vp, vp, ctypes.c_int32, vp]
            lib.mcm_solve_algo.restype = ctypes.c_int
            lib.mcm_solve_noalloc.argtypes = [i32p, ctypes.c_int32, vp, vp, vp]
            lib.mcm_solve_noalloc.restype = ctypes.c_int
            i64p = ctypes.POINTER(ctypes.c_int64)
            lib.mcm_solve_batched.argtypes = [ctypes.c_int32, i32p, i64p, i32p, i64p, vp, vp, vp]
            lib.mcm_solve_batched.restype = ctypes.c_int
            lib.mcm_chain_create.argtypes = [i32p, ctypes.c_int32, vp, ctypes.POINTER(vp)]
            lib.mcm_chain_create.restype = ctypes.c_int
            lib.mcm_chain_solve.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
            lib.mcm_chain_solve.restype = ctypes.c_int
            lib.mcm_chain_n.argtypes = [vp]
            lib.mcm_chain_n.restype = ctypes.c_int32
            lib.mcm_chain_destroy.argtypes = [vp, vp]
            lib.mcm_chain_destroy.restype = None
            i64p = ctypes.POINTER(ctypes.c_int64)
            lib.mcm_plan_create.argtypes = [ctypes.c_int32, i32p, i64p, i64p, ctypes.c_int32,
                                            ctypes.POINTER(vp)]
            lib.mcm_plan_create.restype = ctypes.c_int
            lib.mcm_plan_solve.argtypes = [vp, i32p, vp, vp, vp]
            lib.mcm_plan_solve.restype = ctypes.c_int
            lib.mcm_plan_autotune.argtypes = [vp, i32p, vp, vp, vp, ctypes.POINTER(ctypes.c_int32)]
            lib.mcm_plan_autotune.restype = ctypes.c_int
            lib.mcm_plan_config.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int32)] * 3
            lib.mcm_plan_config.restype = ctypes.c_int
            lib.mcm_plan_set_config.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
            lib.mcm_plan_set_config.restype = ctypes.c_int
            lib.mcm_plan_candidates.argtypes = [vp, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_float),
                                                ctypes.POINTER(ctypes.c_int32)]
            lib.mcm_plan_candidates.restype = ctypes.c_int
            lib.mcm_plan_graph_create.argtypes = [vp, vp, vp, vp]
            lib.mcm_plan_graph_create.restype = ctypes.c_int
            lib.mcm_plan_graph_solve.argtypes = [vp, i32p, vp]
            lib.mcm_plan_graph_solve.restype = ctypes.c_int
            lib.mcm_plan_destroy.argtypes = [vp]
            lib.mcm_plan_destroy.restype = None
            lib.mcm_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, vp,
                                              ctypes.POINTER(vp)]
            lib.mcm_server_create.restype = ctypes.c_int
            lib.mcm_server_submit.argtypes = [vp, i32p, ctypes.c_int32, ctypes.c_uint64]
            lib.mcm_server_submit.restype = ctypes.c_int
            lib.mcm_server_poll.argtypes = [vp, ctypes.POINTER(RequestInfo), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]
            lib.mcm_server_poll.restype = ctypes.c_int
            lib.mcm_server_release.argtypes = [vp, ctypes.c_uint64]
            lib.mcm_server_release.restype = ctypes.c_int
            lib.mcm_server_request_bytes.argtypes = [i32p, ctypes.c_int32]
            lib.mcm_server_request_bytes.restype = ctypes.c_size_t
            lib.mcm_server_stats.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int64)] * 5
            lib.mcm_server_stats.restype = ctypes.c_int
            lib.mcm_server_destroy.argtypes = [vp]
            lib.mcm_server_destroy.restype = None
            lib.mcm_clock_now.argtypes = []
            lib.mcm_clock_now.restype = ctypes.c_double
            lib.mcm_profile_enable.argtypes = [ctypes.c_int32]
            lib.mcm_profile_enable.restype = None
            lib.mcm_profile_enable_mask.argtypes = [ctypes.c_uint32]
            lib.mcm_profile_enable_mask.restype = None
            lib.mcm_profile_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_double)]
            lib.mcm_profile_read.restype = ctypes.c_int
            lib.mcm_parens_length.argtypes = [ctypes.c_int32]
            lib.mcm_parens_length.restype = ctypes.c_int64
            lib.mcm_parenthesize.argtypes = [i32p, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
            lib.mcm_parenthesize.restype = ctypes.c_int
            lib.mcm_parenthesize_batched.argtypes = [ctypes.c_int32, i32p, i64p, i32p, i64p, vp,
                                                     i64p, vp, vp, vp, vp]
            lib.mcm_parenthesize_batched.restype = ctypes.c_int
            lib.mcm_sdp_solve.argtypes = [i32p, ctypes.c_int32, ctypes.c_int32, vp,
                                          ctypes.c_int32, vp]
            lib.mcm_sdp_solve.restype = ctypes.c_int
            lib.mcm_obst_solve.argtypes = [i32p, i32p, ctypes.c_int32, vp, vp, vp]
            lib.mcm_obst_solve.restype = ctypes.c_int
            lib.mcm_obst_solve_algo.argtypes = [i32p, i32p, ctypes.c_int32, vp, vp,
                                                ctypes.c_int32, vp]
            lib.mcm_obst_solve_algo.restype = ctypes.c_int
            _lib = lib
    return _lib


def status_string(status: int) -> str:
    return load().mcm_status_string(int(status)).decode()


def version() -> int:
    return int(load().mcm_version())


def _dims(p) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(p, dtype=np.int32))
    if a.ndim != 1:
        raise ValueError("p must be one-dimensional")
    return a


def _p_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def check_chain(p) -> int:
    """mcm_check_chain status for p[0..n] (host only)."""
    a = _dims(p)
    return int(load().mcm_check_chain(_p_ptr(a), a.size - 1))


def select_algo(p) -> int:
    a = _dims(p)
    return int(load().mcm_select_algo(_p_ptr(a), a.size - 1))


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def solve_into(p, m, s, algo: int | str = ALGO_AUTO, stream=None) -> None:
    """Enqueue the solve of chain p into preallocated device tensors.

    m: int64 CUDA tensor with n*n elements, s: int32 CUDA tensor with n*n
    elements (both contiguous).  Returns once enqueued on `stream`
    (default: torch's current stream).
    """
    import torch
    a = _dims(p)
    n = a.size - 1
    if isinstance(algo, str):
        algo = ALGOS[algo]
    if not (m.is_cuda and s.is_cuda and m.dtype == torch.int64 and s.dtype == torch.int32):
        raise TypeError("m must be a CUDA int64 tensor and s a CUDA int32 tensor")
    if not (m.is_contiguous() and s.is_contiguous()) or m.numel() < n * n or s.numel() < n * n:
        raise ValueError("m and s must be contiguous with at least n*n elements")
    st = load().mcm_solve_algo(_p_ptr(a), n, ctypes.c_void_p(m.data_ptr()),
                               ctypes.c_void_p(s.data_ptr()), int(algo),
                               ctypes.c_void_p(_stream_handle(stream)))
    if st != OK:
        raise MCMError(st, "mcm_solve_algo")


def solve_noalloc_into(p, m, s, stream=None) -> None:
    """mcm_solve_noalloc: the solve of chain p into preallocated device
    tensors (as solve_into) with no device allocation by the library; its
    workspace is the library's fixed per-device array."""
    import torch
    a = _dims(p)
    n = a.size - 1
    if not (m.is_cuda and s.is_cuda and m.dtype == torch.int64 and s.dtype == torch.int32):
        raise TypeError("m must be a CUDA int64 tensor and s a CUDA int32 tensor")
    if not (m.is_contiguous() and s.is_contiguous()) or m.numel() < n * n or s.numel() < n * n:
        raise ValueError("m and s must be contiguous with at least n*n elements")
    st = load().mcm_solve_noalloc(_p_ptr(a), n, ctypes.c_void_p(m.data_ptr()),
                                  ctypes.c_void_p(s.data_ptr()),
                                  ctypes.c_void_p(_stream_handle(stream)))
    if st != OK:
        raise MCMError(st, "mcm_solve_noalloc")


def solve(p, algo: int | str = ALGO_AUTO, device="cuda", stream=None):
    """Solve chain p; returns (m, s) as (n, n) CUDA tensors (int64, int32).

    The work is enqueued on `stream`; synchronise before reading on the host.
    """
    import torch
    a = _dims(p)
    n = a.size - 1
    m = torch.empty((max(n, 0), max(n, 0)), dtype=torch.int64, device=device)
    s = torch.empty((max(n, 0), max(n, 0)), dtype=torch.int32, device=device)
    solve_into(a, m, s, algo=algo, stream=stream)
    return m, s


def solve_batched_into(ns, p_off, p_all, tab_off, m_all, s_all, stream=None) -> None:
    """Enqueue mcm_solve_batched: chain b has ns[b] matrices, dims
    p_all[p_off[b] : p_off[b] + ns[b] + 1], and writes its n*n tables at
    element offset tab_off[b] of the flat device tensors m_all (int64) and
    s_all (int32)."""
    import torch
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    p_off = np.ascontiguousarray(np.asarray(p_off, dtype=np.int64))
    p_all = np.ascontiguousarray(np.asarray(p_all, dtype=np.int32))
    tab_off = np.ascontiguousarray(np.asarray(tab_off, dtype=np.int64))
    count = ns.size
    if not (p_off.size == count and tab_off.size == count):
        raise ValueError("ns, p_off and tab_off must have one entry per chain")
    if not (m_all.is_cuda and s_all.is_cuda and m_all.dtype == torch.int64 and
            s_all.dtype == torch.int32 and m_all.is_contiguous() and s_all.is_contiguous()):
        raise TypeError("m_all / s_all must be contiguous CUDA int64 / int32 tensors")
    if count:
        if np.any(ns < 1) or np.any(p_off < 0) or np.any(tab_off < 0):
            raise ValueError("n >= 1 and non-negative offsets required")
        if int(np.max(p_off + ns + 1)) > p_all.size:
            raise ValueError("p_all too short for the given offsets")
        need = int(np.max(tab_off + ns.astype(np.int64) ** 2))
        if m_all.numel() < need or s_all.numel() < need:
            raise ValueError("m_all / s_all too small for the given table offsets")
    i64 = ctypes.POINTER(ctypes.c_int64)
    st = load().mcm_solve_batched(count, _p_ptr(ns), p_off.ctypes.data_as(i64), _p_ptr(p_all),
                                  tab_off.ctypes.data_as(i64), ctypes.c_void_p(m_all.data_ptr()),
                                  ctypes.c_void_p(s_all.data_ptr()),
                                  ctypes.c_void_p(_stream_handle(stream)))
    if st != OK:
        raise MCMError(st, "mcm_solve_batched")


def parens_length(n: int) -> int:
    """mcm_parens_length: characters of the parenthesized text of n matrices."""
    return int(load().mcm_parens_length(int(n)))


def _ptr_or_null(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def parenthesize_into(s, n: int, p=None, lo=None, hi=None, cost=None, text=None,
                      stream=None) -> None:
    """Enqueue mcm_parenthesize for the n x n split table s (CUDA int32).

    lo, hi: CUDA int32 tensors of n-1 elements (or both None); cost: CUDA
    int64 tensor of one element (needs p); text: CUDA uint8 tensor of
    parens_length(n)+1 bytes.  Any output may be None.
    """
    import torch
    if not (s.is_cuda and s.dtype == torch.int32 and s.is_contiguous() and s.numel() >= n * n):
        raise TypeError("s must be a contiguous CUDA int32 tensor of n*n elements")
    for t, dt, need in ((lo, torch.int32, n - 1), (hi, torch.int32, n - 1),
                        (cost, torch.int64, 1), (text, torch.uint8, parens_length(n) + 1)):
        if t is not None and not (t.is_cuda and t.dtype == dt and t.is_contiguous() and
                                  t.numel() >= need):
            raise TypeError("output tensor of the wrong type or size")
    a = _dims(p) if p is not None else None
    if a is not None and a.size != n + 1:
        raise ValueError("p must have n+1 entries")
    st = load().mcm_parenthesize(_p_ptr(a) if a is not None else None, int(n),
                                 ctypes.c_void_p(s.data_ptr()), _ptr_or_null(lo),
                                 _ptr_or_null(hi), _ptr_or_null(cost), _ptr_or_null(text),
                                 ctypes.c_void_p(_stream_handle(stream)))
    if st != OK:
        raise MCMError(st, "mcm_parenthesize")


def parenthesize(s, p=None, stream=None):
    """Tree of the split table s (n x n CUDA int32) on the device.

    Returns (lo, hi, cost, text): lo/hi CUDA int32 tensors (n-1), cost an
    int (None without p), text a str.  Synchronises the stream to read
    cost and text.
    """
    import torch
    n = int(s.shape[0])
    dev = s.device
    lo = torch.empty(max(n - 1, 0), dtype=torch.int32, device=dev)
    hi = torch.empty(max(n - 1, 0), dtype=torch.int32, device=dev)
    cost = torch.empty(1, dtype=torch.int64, device=dev) if p is not None else None
    text = torch.empty(parens_length(n) + 1, dtype=torch.uint8, device=dev)
    parenthesize_into(s, n, p=p, lo=lo if n > 1 else None, hi=hi if n > 1 else None,
                      cost=cost, text=text, stream=stream)
    raw = text.cpu().numpy().tobytes()
    return (lo, hi, int(cost.item()) if cost is not None else None,
            raw[:raw.index(b"\0")].decode("ascii"))


def parenthesize_batched_into(ns, tab_off, s_all, node_off, lo_all, hi_all, p_off=None,
                              p_all=None, cost_all=None, stream=None) -> None:
    """Enqueue mcm_parenthesize_batched (offsets as in solve_batched_into;
    chain b's products at node_off[b] of lo_all / hi_all)."""
    import torch
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    tab_off = np.ascontiguousarray(np.asarray(tab_off, dtype=np.int64))
    node_off = np.ascontiguousarray(np.asarray(node_off, dtype=np.int64))
    count = ns.size
    if not (tab_off.size == count and node_off.size == count):
        raise ValueError("ns, tab_off and node_off must have one entry per chain")
    for t, dt in ((s_all, torch.int32), (lo_all, torch.int32), (hi_all, torch.int32)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise TypeError("s_all / lo_all / hi_all must be contiguous CUDA int32 tensors")
    if count:
        if np.any(ns < 1) or np.any(tab_off < 0) or np.any(node_off < 0):
            raise ValueError("n >= 1 and non-negative offsets required")
        if int(np.max(tab_off + ns.astype(np.int64) ** 2)) > s_all.numel():
            raise ValueError("s_all too small for the given table offsets")
        if int(np.max(node_off + ns - 1)) > min(lo_all.numel(), hi_all.numel()):
            raise ValueError("lo_all / hi_all too small for the given node offsets")
    i64 = ctypes.POINTER(ctypes.c_int64)
    pa = po = None
    if cost_all is not None:
        if p_off is None or p_all is None:
            raise ValueError("cost_all needs p_off and p_all")
        if not (cost_all.is_cuda and cost_all.dtype == torch.int64 and
                cost_all.is_contiguous() and cost_all.numel() >= count):
            raise TypeError("cost_all must be a contiguous CUDA int64 tensor of count entries")
        po = np.ascontiguousarray(np.asarray(p_off, dtype=np.int64))
        pa = np.ascontiguousarray(np.asarray(p_all, dtype=np.int32))
        if po.size != count or (count and int(np.max(po + ns + 1)) > pa.size):
            raise ValueError("p_off / p_all do not cover the chains")
    st = load().mcm_parenthesize_batched(
        count, _p_ptr(ns), po.ctypes.data_as(i64) if po is not None else None,
        _p_ptr(pa) if pa is not None else None, tab_off.ctypes.data_as(i64),
        ctypes.c_void_p(s_all.data_ptr()), node_off.ctypes.data_as(i64),
        ctypes.c_void_p(lo_all.data_ptr()), ctypes.c_void_p(hi_all.data_ptr()),
        _ptr_or_null(cost_all), ctypes.c_void_p(_stream_handle(stream)))
    if st != OK:
        raise MCMError(st, "mcm_parenthesize_batched")


def sdp_solve_into(offsets, st, op: str = "min", stream=None) -> None:
    """Enqueue mcm_sdp_solve: st is a contiguous CUDA int32 tensor of n
    elements whose first offsets[0] entries hold the preset values."""
    import torch
    a = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
    if a.ndim != 1:
        raise ValueError("offsets must be one-dimensional")
    if not (st.is_cuda and st.dtype == torch.int32 and st.is_contiguous()):
        raise TypeError("st must be a contiguous CUDA int32 tensor")
    rc = load().mcm_sdp_solve(_p_ptr(a), a.size, SDP_OPS[op], ctypes.c_void_p(st.data_ptr()),
                              st.numel(), ctypes.c_void_p(_stream_handle(stream)))
    if rc != OK:
        raise MCMError(rc, "mcm_sdp_solve")


def obst_solve(p, q, algo: int | str = ALGO_AUTO, device="cuda", stream=None):
    """Optimal binary search tree (mcm_obst_solve_algo): returns the
    (n+1) x (n+1) CUDA tensors (e int64, root int32); enqueued on `stream`."""
    import torch
    pa = np.ascontiguousarray(np.asarray(p, dtype=np.int32))
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.int32))
    n = pa.size
    if qa.size != n + 1:
        raise ValueError("need n+1 gap weights")
    e = torch.empty((n + 1, n + 1), dtype=torch.int64, device=device)
    root = torch.empty((n + 1, n + 1), dtype=torch.int32, device=device)
    if isinstance(algo, str):
        algo = ALGOS[algo]
    rc = load().mcm_obst_solve_algo(_p_ptr(pa) if n else None, _p_ptr(qa), n,
                                    ctypes.c_void_p(e.data_ptr()),
                                    ctypes.c_void_p(root.data_ptr()), int(algo),
                                    ctypes.c_void_p(_stream_handle(stream)))
    if rc != OK:
        raise MCMError(rc, "mcm_obst_solve_algo")
    return e, root


def node_offsets(ns) -> np.ndarray:
    """Packed offsets of n-1 product entries per chain, one after another."""
    ns = np.asarray(ns, dtype=np.int64)
    off = np.zeros(ns.size, dtype=np.int64)
    if ns.size > 1:
        off[1:] = np.cumsum(ns[:-1] - 1)
    return off


def table_offsets(ns) -> np.ndarray:
    """Packed element offsets of n*n tables, one after another."""
    ns = np.asarray(ns, dtype=np.int64)
    off = np.zeros(ns.size, dtype=np.int64)
    if ns.size > 1:
        off[1:] = np.cumsum(ns[:-1] ** 2)
    return off


class Chain:
    """A validated chain whose dimensions live in device memory
    (mcm_chain_create); solve it repeatedly with :meth:`solve_into`."""

    def __init__(self, p, stream=None):
        a = _dims(p)
        self.n = a.size - 1
        h = ctypes.c_void_p()
        st = load().mcm_chain_create(_p_ptr(a), self.n, ctypes.c_void_p(_stream_handle(stream)),
                                     ctypes.byref(h))
        if st != OK:
            raise MCMError(st, "mcm_chain_create")
        self._h = h

    def solve_into(self, m, s, algo: int | str = ALGO_AUTO, stream=None) -> None:
        import torch
        if isinstance(algo, str):
            algo = ALGOS[algo]
        n = self.n
        if not (m.is_cuda and s.is_cuda and m.dtype == torch.int64 and s.dtype == torch.int32):
            raise TypeError("m must be a CUDA int64 tensor and s a CUDA int32 tensor")
        if not (m.is_contiguous() and s.is_contiguous()) or m.numel() < n * n or \
                s.numel() < n * n:
            raise ValueError("m and s must be contiguous with at least n*n elements")
        st = load().mcm_chain_solve(self._h, int(algo), ctypes.c_void_p(m.data_ptr()),
                                    ctypes.c_void_p(s.data_ptr()),
                                    ctypes.c_void_p(_stream_handle(stream)))
        if st != OK:
            raise MCMError(st, "mcm_chain_solve")

    def close(self, stream=None) -> None:
        if self._h:
            load().mcm_chain_destroy(self._h, ctypes.c_void_p(_stream_handle(stream)))
            self._h = None


class Plan:
    """A batched plan (mcm_plan_create) for a fixed batch shape: chain b has
    ns[b] matrices, dims at p_all[p_off[b] : p_off[b] + ns[b] + 1], tables at
    element offset tab_off[b]; every dim at most max_dim.  Solve it with
    :meth:`solve_into` for any dims of that shape."""

    def __init__(self, ns, p_off, tab_off, max_dim: int):
        self.ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
        self.p_off = np.ascontiguousarray(np.asarray(p_off, dtype=np.int64))
        self.tab_off = np.ascontiguousarray(np.asarray(tab_off, dtype=np.int64))
        if not (self.p_off.size == self.ns.size and self.tab_off.size == self.ns.size):
            raise ValueError("ns, p_off and tab_off must have one entry per chain")
        count = self.ns.size
        self.p_len = int(np.max(self.p_off + self.ns + 1)) if count else 0
        self.need = int(np.max(self.tab_off + self.ns.astype(np.int64) ** 2)) if count else 0
        i64 = ctypes.POINTER(ctypes.c_int64)
        h = ctypes.c_void_p()
        st = load().mcm_plan_create(count, _p_ptr(self.ns), self.p_off.ctypes.data_as(i64),
                                    self.tab_off.ctypes.data_as(i64), int(max_dim),
                                    ctypes.byref(h))
        if st != OK:
            raise MCMError(st, "mcm_plan_create")
        self._h = h

    def _args(self, p_all, m_all, s_all):
        import torch
        p_all = np.ascontiguousarray(np.asarray(p_all, dtype=np.int32))
        if p_all.size < self.p_len:
            raise ValueError("p_all too short for the plan's offsets")
        if not (m_all.is_cuda and s_all.is_cuda and m_all.dtype == torch.int64 and
                s_all.dtype == torch.int32 and m_all.is_contiguous() and s_all.is_contiguous()):
            raise TypeError("m_all / s_all must be contiguous CUDA int64 / int32 tensors")
        if m_all.numel() < self.need or s_all.numel() < self.need:
            raise ValueError("m_all / s_all too small for the plan's table offsets")
        return p_all

    def solve_into(self, p_all, m_all, s_all, stream=None) -> None:
        p_all = self._args(p_all, m_all, s_all)
        st = load().mcm_plan_solve(self._h, _p_ptr(p_all), ctypes.c_void_p(m_all.data_ptr()),
                                   ctypes.c_void_p(s_all.data_ptr()),
                                   ctypes.c_void_p(_stream_handle(stream)))
        if st != OK:
            raise MCMError(st, "mcm_plan_solve")

    def autotune(self, p_all, m_all, s_all, stream=None) -> int:
        """Time every configuration (tile edge, closure threshold) on these
        inputs and keep the fastest; returns its index in candidates()."""
        p_all = self._args(p_all, m_all, s_all)
        choice = ctypes.c_int32(0)
        st = load().mcm_plan_autotune(self._h, _p_ptr(p_all), ctypes.c_void_p(m_all.data_ptr()),
                                      ctypes.c_void_p(s_all.data_ptr()),
                                      ctypes.c_void_p(_stream_handle(stream)),
                                      ctypes.byref(choice))
        if st != OK:
            raise MCMError(st, "mcm_plan_autotune")
        return int(choice.value)

    def graph_create(self, m_all, s_all, stream=None) -> None:
        """Record the plan's solve into a HIP graph for these outputs."""
        import torch
        self._args(np.ones(self.p_len, dtype=np.int32), m_all, s_all)
        if stream is None:
            stream = torch.cuda.current_stream()
        st = load().mcm_plan_graph_create(self._h, ctypes.c_void_p(m_all.data_ptr()),
                                          ctypes.c_void_p(s_all.data_ptr()),
                                          ctypes.c_void_p(_stream_handle(stream)))
        if st != OK:
            raise MCMError(st, "mcm_plan_graph_create")

    def graph_solve(self, p_all, stream=None) -> None:
        """One solve by replaying the recorded graph with new dims."""
        p_all = np.ascontiguousarray(np.asarray(p_all, dtype=np.int32))
        if p_all.size < self.p_len:
            raise ValueError("p_all too short for the plan's offsets")
        st = load().mcm_plan_graph_solve(self._h, _p_ptr(p_all),
                                         ctypes.c_void_p(_stream_handle(stream)))
        if st != OK:
            raise MCMError(st, "mcm_plan_graph_solve")

    def config(self) -> dict:
        """{'tile_edge', 'pair_min_blocks', 'source'} of the configuration in use."""
        v = [ctypes.c_int32(0) for _ in range(3)]
        st = load().mcm_plan_config(self._h, *[ctypes.byref(x) for x in v])
        if st != OK:
            raise MCMError(st, "mcm_plan_config")
        return {"tile_edge": v[0].value, "pair_min_blocks": v[1].value,
                "source": PLAN_SOURCES[v[2].value]}

    def set_config(self, tile_edge: int, pair_min_blocks: int = 0) -> None:
        st = load().mcm_plan_set_config(self._h, int(tile_edge), int(pair_min_blocks))
        if st != OK:
            raise MCMError(st, "mcm_plan_set_config")

    def candidates(self) -> list:
        """[{'tile_edge', 'pair_min_blocks', 'ms'}] in autotune order (ms from
        the last autotune, None if never timed)."""
        cnt = ctypes.c_int32(0)
        lib = load()
        st = lib.mcm_plan_candidates(self._h, 0, None, None, None, ctypes.byref(cnt))
        if st != OK:
            raise MCMError(st, "mcm_plan_candidates")
        k = cnt.value
        te = (ctypes.c_int32 * max(k, 1))()
        pm = (ctypes.c_int32 * max(k, 1))()
        ms = (ctypes.c_float * max(k, 1))()
        st = lib.mcm_plan_candidates(self._h, k, te, pm, ms, ctypes.byref(cnt))
        if st != OK:
            raise MCMError(st, "mcm_plan_candidates")
        return [{"tile_edge": te[i], "pair_min_blocks": pm[i],
                 "ms": None if ms[i] < 0 else float(ms[i])} for i in range(k)]

    def close(self) -> None:
        if self._h:
            load().mcm_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def server_request_bytes(p) -> int:
    """Arena bytes the server holds for a request of chain p (0 if invalid)."""
    a = _dims(p)
    return int(load().mcm_server_request_bytes(_p_ptr(a), a.size - 1))


def clock_now() -> float:
    """Seconds on the steady clock the server's timestamps use."""
    return float(load().mcm_clock_now())


_hip = None


def copy_device_to_host(dst: np.ndarray, src_ptr: int) -> None:
    """Synchronous hipMemcpy of dst.nbytes from device address src_ptr."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst.ctypes.data), ctypes.c_void_p(src_ptr),
                        dst.nbytes, 2)  # hipMemcpyDeviceToHost
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


class Server:
    """mcm_server: continuous batching of chain solves on one device."""

    def __init__(self, mem_budget: int, max_slots: int = 256, stream=None):
        h = ctypes.c_void_p()
        st = load().mcm_server_create(int(mem_budget), int(max_slots),
                                      ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h))
        if st != OK:
            raise MCMError(st, "mcm_server_create")
        self._h = h
        self._buf = (RequestInfo * 256)()

    def submit(self, p, tag: int) -> None:
        a = _dims(p)
        st = load().mcm_server_submit(self._h, _p_ptr(a), a.size - 1, ctypes.c_uint64(tag))
        if st != OK:
            raise MCMError(st, "mcm_server_submit")

    def poll(self) -> list:
        """Completed requests (RequestInfo copies), oldest first."""
        out = []
        cnt = ctypes.c_int32(0)
        while True:
            st = load().mcm_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(cnt))
            if st != OK:
                raise MCMError(st, "mcm_server_poll")
            out.extend(RequestInfo.from_buffer_copy(self._buf[i]) for i in range(cnt.value))
            if cnt.value < len(self._buf):
                return out

    def fetch(self, info: RequestInfo):
        """Copy a completed request's tables to host numpy arrays."""
        n = info.n
        m = np.empty((n, n), dtype=np.int64)
        s = np.empty((n, n), dtype=np.int32)
        copy_device_to_host(m, info.m)
        copy_device_to_host(s, info.s)
        return m, s

    def release(self, tag: int) -> None:
        st = load().mcm_server_release(self._h, ctypes.c_uint64(tag))
        if st != OK:
            raise MCMError(st, "mcm_server_release")

    def stats(self) -> dict:
        v = [ctypes.c_int64(0) for _ in range(5)]
        st = load().mcm_server_stats(self._h, *[ctypes.byref(x) for x in v])
        if st != OK:
            raise MCMError(st, "mcm_server_stats")
        return dict(zip(["queued", "active", "completed", "iterations", "bytes_in_use"],
                        [x.value for x in v]))

    def close(self) -> None:
        if self._h:
            load().mcm_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def profile_enable(on: bool = True, classes=None, serial: bool = False) -> None:
    """Time every kernel class (or only those listed in `classes`).
    serial: single-chain tiled solves run the serial schedule meanwhile
    (MCM_PROFILE_SERIAL), so each timed launch has the device alone."""
    if classes is None and not serial:
        load().mcm_profile_enable(1 if on else 0)
        return
    mask = 0
    for c in (range(5) if classes is None else classes):
        mask |= 1 << int(c)
    if serial:
        mask |= PROFILE_SERIAL
    load().mcm_profile_enable_mask(mask if on else 0)


def profile_read(kernel_class: int) -> dict:
    """{'ms', 'launches', 'split_evals'} accumulated for a kernel class."""
    ms = ctypes.c_double(0.0)
    nl = ctypes.c_int64(0)
    ev = ctypes.c_double(0.0)
    st = load().mcm_profile_read(int(kernel_class), ctypes.byref(ms), ctypes.byref(nl),
                                 ctypes.byref(ev))
    if st != OK:
        raise MCMError(st, "mcm_profile_read")
    return {"ms": ms.value, "launches": nl.value, "split_evals": ev.value}
