"""MI355X-native matrix-chain-multiplication DP solver (gfx950 HIP kernels).

The solver fills the exact int64 cost table m and the int32 split table s
of the matrix-chain-multiplication DP (Section IV of the paper) on one GPU,
behind the C ABI declared in ``include/mcm.h``.  This package holds the HIP
sources (``csrc/``), their build step (``build``), the ctypes binding
(``binding``) and the seeded workload generators (``workloads``).

Importing the package loads nothing; the library is loaded on first use.
"""
from __future__ import annotations

__all__ = ["solve", "solve_into", "check_chain", "select_algo", "MCMError", "Chain",
           "solve_batched_into", "table_offsets", "Server",
           "profile_enable", "profile_read", "ALGOS"]


def __getattr__(name):
    if name in __all__:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
