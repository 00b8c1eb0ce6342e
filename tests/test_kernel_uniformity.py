"""Static check of the read-back walk kernel (no GPU): the compiler's
uniformity analysis must find no loop with a divergent exit in k_paren
other than its three per-thread loops (the table and count
initialisations and the final cost sum).  The queue loop and the walks must stay wave-uniform: a lane-0
branch around the queue-slot claim once let the compiler send the other
lanes back to a stale slot, and the kernel never finished."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2008_01938_amd", "csrc", "k_paren.hip")


def _tool(name):
    for cand in (shutil.which(name), f"/opt/rocm/bin/{name}", f"/opt/rocm/llvm/bin/{name}"):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.mark.skipif(_tool("hipcc") is None or _tool("opt") is None, reason="ROCm tools missing")
def test_walk_kernel_loops_are_uniform(tmp_path):
    from paper_2008_01938_amd import build
    ll = tmp_path / "k_paren.ll"
    flags = [f for f in build.HIPCC_FLAGS if f != "-fPIC"]
    subprocess.run([_tool("hipcc"), *flags, f"-I{os.path.dirname(SRC)}", "--cuda-device-only",
                    "-emit-llvm", "-S", "-o", str(ll), SRC], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    res = subprocess.run([_tool("opt"), "-mtriple=amdgcn-amd-amdhsa", "-mcpu=gfx950",
                          "-passes=print<uniformity>", "-disable-output", str(ll)],
                         capture_output=True, text=True, check=True)
    text = res.stderr + res.stdout
    # One report per function; keep the walk kernels' reports.
    reports = re.split(r"(?=UniformityInfo for function)", text)
    walk = [r for r in reports if re.search(r"'_Z\S*k_paren\S*EEEv", r.splitlines()[0] if r else "")]
    assert len(walk) == 2, "expected the two k_paren instantiations"
    for r in walk:
        m = re.search(r"CYCLES WITH DIVERGENT EXIT:\n((?:  depth=.*\n)*)", r)
        cycles = m.group(1).strip().splitlines() if m else []
        # the two grid-stride initialisation loops and the final cost loop
        assert len(cycles) <= 3, cycles
        assert all(c.strip().startswith("depth=1") for c in cycles), cycles
