"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers are built into ``tests/sanitize/_build`` and run:

* ``oracle_checks`` -- the C oracle (``oracle/mcm_oracle.c``) with gcc's
  sanitizers: fills, the cell checker and validation edge cases;
* ``host_checks`` -- the library's host code (validation, batched range
  checks and the tiled planner) with hipcc, sanitizers on the host side
  only; its kernels are compiled but never launched, so no GPU is needed.

A sanitizer report aborts the driver, which fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(HERE, "_build")
CSRC = os.path.join(ROOT, "paper_2008_01938_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, timeout):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=ENV)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed:\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.fixture(scope="module")
def outdir():
    os.makedirs(OUT, exist_ok=True)
    return OUT


def test_oracle_under_sanitizers(outdir):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = os.path.join(outdir, "oracle_checks")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-o", exe, os.path.join(HERE, "oracle_checks.c"),
          os.path.join(ROOT, "oracle", "mcm_oracle.c")], timeout=300)
    r = _run([exe], timeout=300)
    assert "oracle checks passed" in r.stdout


def test_library_host_code_under_sanitizers(outdir):
    from paper_2008_01938_amd import build
    exe = os.path.join(outdir, "host_checks")
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    flags = [f"--offload-arch={build.ARCH}", "-O1", "-g", "-std=c++17", "-fno-honor-nans",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{os.path.join(ROOT, 'include')}",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]
    _run([build.hipcc(), *flags, "-o", exe, os.path.join(HERE, "host_checks.cpp"), *srcs],
         timeout=900)
    r = _run([exe], timeout=600)
    assert "host checks passed" in r.stdout
