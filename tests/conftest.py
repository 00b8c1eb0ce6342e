"""Shared pytest configuration.

Tests marked ``gpu`` need an AMD Instinct GPU (gfx950) and the built HIP
library; everything else runs on the CPU.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a gfx950 GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running case")


@pytest.fixture(scope="session")
def n8192_oracle():
    """The oracle's whole tables for the n = 8192 benchmark chain (dims
    uniform in [1, 1024], seed 2), filled once on every host thread."""
    import oracle
    from paper_2008_01938_amd import workloads
    p = workloads.single_n8192()
    print("[cpu] oracle fill n=8192 on all host threads", flush=True)
    m, s = oracle.fill(p, threads=oracle.default_threads())
    return p, m, s
