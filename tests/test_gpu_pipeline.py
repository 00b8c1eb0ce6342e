"""The pipeline of Fig. 8 with stalls (MCM_ALGO_PIPELINE), an ablation:
bit-exact against the oracle like the other paths."""
import sys

import numpy as np
import pytest

import oracle
from paper_2008_01938_amd import binding, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()


@pytest.mark.parametrize("n,seed,hi", [(1, 0, 9), (2, 1, 9), (3, 2, 9), (17, 3, 50), (64, 4, 1024),
                                       (65, 5, 2), (200, 6, 1024)])
def test_against_oracle(n, seed, hi):
    import torch
    p = workloads.uniform_dims(n, 1, hi, seed)
    print(f"[gpu] pipeline n={n}", flush=True)
    sys.stdout.flush()
    m, s = binding.solve(p, algo="pipeline")
    torch.cuda.synchronize()
    om, os_ = oracle.fill(p)
    assert np.array_equal(m.cpu().numpy(), om) and np.array_equal(s.cpu().numpy(), os_)


def test_size_limit():
    with pytest.raises(binding.MCMError):
        binding.solve(workloads.uniform_dims(1026, 1, 9, 0), algo="pipeline")
