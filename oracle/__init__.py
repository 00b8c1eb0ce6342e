"""CPU oracle for the matrix-chain-multiplication DP table.

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only code allowed to import it.  It
shares no code with the GPU library (``paper_2008_01938_amd``), and neither
side imports the other; both take their inputs from the seeded generators
in ``paper_2008_01938_amd.workloads``, which hold none of the method's
arithmetic.

Two independent implementations live here:

* ``mcm_oracle.c`` (wrapped by :func:`fill`): the textbook recurrence the
  paper's Section IV refers to, as a plain int64 triple loop in diagonal
  order (Fig. 5), smallest split on ties.
* :mod:`oracle.linear`: the paper's own formulation -- the triangular table
  linearised into a 1-D array ``ST`` in diagonal order and every element
  computed by Eq. (2) from its operand pairs -- in pure Python, for small n.
* :mod:`oracle.paren`: the optimal product order read back from a split
  table by the textbook recursion (tree, cost and parenthesized text).

Neither is trusted on its own: ``tests/test_oracle.py`` pins both against
brute-force enumeration of parenthesizations, closed forms, invariants and
the paper's worked n=5 indexing example.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcm_oracle.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD_DIR, "libmcm_oracle.so")

OK, INVALID, OVERFLOW = 0, 1, 2

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP enabled); return the .so path."""
    os.makedirs(_BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i64p = ctypes.POINTER(ctypes.c_int64)
            lib.mcm_oracle_validate.argtypes = [i32p, ctypes.c_int32]
            lib.mcm_oracle_validate.restype = ctypes.c_int
            lib.mcm_oracle_fill.argtypes = [i32p, ctypes.c_int32, i64p, i32p, ctypes.c_int32]
            lib.mcm_oracle_fill.restype = ctypes.c_int
            lib.mcm_oracle_check_cells.argtypes = [i32p, ctypes.c_int32, i64p, i32p, i32p,
                                                  ctypes.c_int64, ctypes.c_int32]
            lib.mcm_oracle_check_cells.restype = ctypes.c_int64
            _lib = lib
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_dims(p) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(p, dtype=np.int32))


def validate(p) -> int:
    """Return OK, INVALID or OVERFLOW for the dimension vector p[0..n]."""
    p = _as_dims(p)
    if p.ndim != 1 or p.size < 2:
        return INVALID
    return int(_load().mcm_oracle_validate(_ptr(p, ctypes.c_int32), p.size - 1))


def fill(p, threads: int = 1):
    """Oracle tables for dims p[0..n]: returns (m int64[n,n], s int32[n,n]).

    Raises ValueError on an invalid chain, OverflowError when
    (n-1)*max(p)^3 >= 2^63.
    """
    p = _as_dims(p)
    if p.ndim != 1 or p.size < 2:
        raise ValueError("p must be a 1-D vector of n+1 >= 2 dimensions")
    n = p.size - 1
    m = np.empty((n, n), dtype=np.int64)
    s = np.empty((n, n), dtype=np.int32)
    rc = _load().mcm_oracle_fill(_ptr(p, ctypes.c_int32), n, _ptr(m, ctypes.c_int64),
                                 _ptr(s, ctypes.c_int32), int(threads))
    if rc == INVALID:
        raise ValueError("invalid chain (n < 1 or a dimension < 1)")
    if rc == OVERFLOW:
        raise OverflowError("(n-1)*max(p)^3 does not fit in int64")
    return m, s


def check_cells(p, m: np.ndarray, s: np.ndarray, cells, threads: int = 1) -> int:
    """Number of cells (i, j) where the table (m, s) breaks the recurrence.

    The recurrence is re-evaluated from the table's own entries at each
    listed cell (i < j).  Zero failures at every cell, plus a zero diagonal,
    means the table is the oracle's by induction.
    """
    p = _as_dims(p)
    n = p.size - 1
    m = np.ascontiguousarray(m, dtype=np.int64)
    s = np.ascontiguousarray(s, dtype=np.int32)
    if m.shape != (n, n) or s.shape != (n, n):
        raise ValueError("tables must be n x n")
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 2))
    bad = _load().mcm_oracle_check_cells(_ptr(p, ctypes.c_int32), n, _ptr(m, ctypes.c_int64),
                                        _ptr(s, ctypes.c_int32), _ptr(cells, ctypes.c_int32),
                                        cells.shape[0], int(threads))
    if bad < 0:
        raise ValueError("invalid arguments to check_cells")
    return int(bad)


def default_threads() -> int:
    """Threads the oracle uses when asked for 'all cores' (sched affinity)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)
