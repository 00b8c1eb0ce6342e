"""Build the gfx950 HIP library ``libmcm.so`` in-tree with hipcc.

    python -m paper_2008_01938_amd.build

compiles every source under ``csrc/`` into ``paper_2008_01938_amd/_lib/``.
hipcc cross-compiles for gfx950 without a GPU present.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libmcm.so")
ROOT = os.path.dirname(HERE)

ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    # wave-wide atomics combine their lanes with a DPP scan (a few
    # instructions) rather than a loop over the active lanes
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=DPP",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # The kernels never produce NaN; without this every fp64 min of a
    # loop-carried value is preceded by a canonicalising v_max_f64.
    "-fno-honor-nans",
    # Keep the compiler from forming packed-fp32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, save_temps_dir: str | None = None) -> str:
    """Compile libmcm.so; returns its path.  Always recompiles."""
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPCC_FLAGS, "-shared", "-o", tmp, *sources()]
    if save_temps_dir:
        os.makedirs(save_temps_dir, exist_ok=True)
        cmd.insert(1, "-save-temps=obj")
        cmd[cmd.index("-o") + 1] = os.path.join(save_temps_dir, "libmcm.so")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=save_temps_dir or LIBDIR)
    if save_temps_dir:
        return os.path.join(save_temps_dir, "libmcm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
