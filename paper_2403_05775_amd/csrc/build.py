"""Compiles the kdss shared library for gfx950 in-tree.

Host sources are built with g++, device sources with hipcc for gfx950 only;
the result is paper_2403_05775_amd/libkdss.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

CSRC = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(CSRC)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libkdss.so")
# a test build whose checked HIP calls can be made to fail on request
OUT_FI = os.path.join(PKG, "libkdss_fi.so")
BUILD = os.path.join(PKG, "_build")
ARCH = "gfx950"

HOST_SOURCES = ["api.cpp", "sct_build.cpp"]
DEVICE_SOURCES = ["kernels.hip", "gnn.hip", "sample.hip", "sct_gpu.hip", "run_static.hip"]
HEADERS = ["kdss_internal.h", os.path.join(ROOT, "include", "kdss.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-Wall"]
# packed fp32 instructions are kept out of every device build
HIP_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _compile(src: str, obj: str, device: bool, defines=()) -> None:
    path = os.path.join(CSRC, src)
    if device:
        cmd = [HIPCC] + COMMON + HIP_FLAGS + list(defines) + ["-c", path, "-o", obj]
    else:
        cmd = ["g++"] + COMMON + ["-pthread", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def build(verbose: bool = False) -> str:
    """Compile every source and link libkdss.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(s, os.path.join(BUILD, s + ".o"), False) for s in HOST_SOURCES]
    jobs += [(s, os.path.join(BUILD, s + ".o"), True) for s in DEVICE_SOURCES]
    fi_obj = os.path.join(BUILD, "kernels_fi.hip.o")
    with cf.ThreadPoolExecutor(max_workers=len(jobs) + 1) as ex:
        futs = [ex.submit(_compile, *j) for j in jobs]
        futs.append(ex.submit(_compile, "kernels.hip", fi_obj, True, ["-DKDSS_FAULT_INJECTION"]))
        for f in futs:
            f.result()
    objs = [j[1] for j in jobs]
    fi_objs = [fi_obj if o.endswith(os.sep + "kernels.hip.o") else o for o in objs]
    for out, ob in ((OUT, objs), (OUT_FI, fi_objs)):
        tmp = out + ".tmp"
        cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + ob + ["-pthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, out)
        if verbose:
            print("built", out)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
