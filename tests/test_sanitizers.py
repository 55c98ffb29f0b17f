"""The host sources (graph checks, clique-tree builder and counter, planner,
C-ABI host calls) and the CPU oracle, built with the address and undefined-
behaviour sanitizers and run on the cases of tests/sanitize/host_driver.cpp.
The device half of the library is replaced by stand-ins that report KDSS_EHIP
(tests/sanitize/device_stubs.cpp).  Any sanitizer report fails the run."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2403_05775_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_sources_and_oracle_under_sanitizers(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include")]
    objs = []
    for src in ("api.cpp", "sct_build.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.check_call(["g++", "-std=c++17", "-pthread"] + SAN + inc + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in ("device_stubs.cpp", "host_driver.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.check_call(["g++", "-std=c++17", "-pthread"] + SAN + inc + ["-c", os.path.join(HERE, src), "-o", o])
        objs.append(o)
    o = str(tmp_path / "oracle.o")
    subprocess.check_call(["gcc", "-std=c11", "-fopenmp"] + SAN + ["-c", os.path.join(ROOT, "oracle", "kdss_oracle.c"),
                                                                    "-o", o])
    objs.append(o)
    exe = str(tmp_path / "host_driver")
    subprocess.check_call(["g++", "-pthread", "-fopenmp"] + SAN + objs + ["-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "ok (0 failed checks)" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
