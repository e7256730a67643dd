"""Build the hpadi shared library (host C++ + HIP kernels for gfx950) in-tree.

    python -m paper_2402_11299_amd.build

produces ``paper_2402_11299_amd/libhpadi.so``.  hipcc cross-compiles the
device code for gfx950 without a GPU present.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhpadi.so")

SOURCES = ["host.cpp", "krylov.cpp", "net.cpp", "kernels.hip", "sweep.hip", "sweep_uni.hip", "sweep_group.hip", "varcoef.hip", "net.hip", "transforms.cpp", "transforms.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-munsafe-fp-atomics",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str, verbose: bool) -> None:
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    cmd = [hipcc(), *flags, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source to an object in parallel, then link libhpadi.so."""
    import concurrent.futures
    import tempfile
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="hpadi_build_") as tmpdir:
        objs = [os.path.join(tmpdir, src + ".o") for src in SOURCES]
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_compile, src, obj, verbose) for src, obj in zip(SOURCES, objs)]:
                f.result()
        tmp = LIB + ".tmp"
        cmd = [hipcc(), *HIPCC_FLAGS, *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libhpadi.so")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
