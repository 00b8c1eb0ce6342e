"""mcm_solve_noalloc against mcm_solve on the GPU: the same bytes, whole
buffers, on consecutive calls that share the fixed device array (each pair
runs a larger chain, then a smaller one), on the fp64-key and int64 tiled
kernels, and at the largest accepted n."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2008_01938_amd import binding, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(p):
    n = len(p) - 1
    m0 = torch.full((n, n), -7, dtype=torch.int64, device="cuda")
    s0 = torch.full((n, n), -9, dtype=torch.int32, device="cuda")
    m1 = torch.full((n, n), -7, dtype=torch.int64, device="cuda")
    s1 = torch.full((n, n), -9, dtype=torch.int32, device="cuda")
    binding.solve_into(p, m0, s0)
    binding.solve_noalloc_into(p, m1, s1)
    torch.cuda.synchronize()
    return (m0, s0), (m1, s1)


@pytest.mark.parametrize("sizes,lo,hi,seed", [
    ((1500, 300), 1, 1024, 21),       # fp64 keys; ragged last tiles
    ((700, 130), 1, 1 << 16, 22),     # beyond the keys' range: int64 kernels
    ((65, 1), 1, 64, 23),             # one full tile plus one matrix, then n = 1
])
def test_noalloc_matches_solve_twice(sizes, lo, hi, seed):
    for n in sizes:
        print(f"[gpu] noalloc n={n} dims [{lo},{hi}] seed={seed}", flush=True)
        p = workloads.uniform_dims(n, lo, hi, seed)
        if n > 1:
            assert (binding.select_algo(p) == binding.ALGO_TILED)
        (m0, s0), (m1, s1) = _both(p)
        assert torch.equal(m0, m1), f"n={n}: m differs"
        assert torch.equal(s0, s1), f"n={n}: s differs"


def test_noalloc_largest_then_small():
    n = binding.NOALLOC_MAX_N
    print(f"[gpu] noalloc n={n} (largest accepted)", flush=True)
    p = workloads.single_n8192()
    assert len(p) - 1 == n
    (m0, s0), (m1, s1) = _both(p)
    assert torch.equal(m0, m1) and torch.equal(s0, s1)
    del m0, s0, m1, s1
    print("[gpu] noalloc n=200 after n=8192", flush=True)
    p = workloads.uniform_dims(200, 1, 1024, 24)
    (m0, s0), (m1, s1) = _both(p)
    assert torch.equal(m0, m1) and torch.equal(s0, s1)


def test_noalloc_rejects_beyond_limit_on_device():
    p = np.ones(binding.NOALLOC_MAX_N + 2, dtype=np.int32)
    m = torch.empty(1, dtype=torch.int64, device="cuda")
    s = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        binding.solve_noalloc_into(p, m, s)   # the binding's own size check
    n = len(p) - 1
    m = torch.empty((n, n), dtype=torch.int64, device="cuda")
    s = torch.empty((n, n), dtype=torch.int32, device="cuda")
    with pytest.raises(binding.MCMError) as e:
        binding.solve_noalloc_into(p, m, s)
    assert e.value.status == binding.ERR_UNSUPPORTED
