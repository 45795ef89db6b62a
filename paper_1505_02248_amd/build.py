"""Build the gfx950 LEM shared library in-tree with hipcc.

Produces ``paper_1505_02248_amd/liblem.so`` from the HIP/C++ sources under
``csrc/``.  Every HIP source is compiled for gfx950 only, with packed-FP32
instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liblem.so")
SOURCES = ["krylov_lem.hip", "krylov_big.hip", "krylov_calib.hip", "dense.hip", "global_krylov.hip", "rosenbrock.hip", "schrodinger.hip",
           "global_static.hip", "kron.hip", "host_op.cpp", "host_krylov.cpp", "host_dense.cpp",
           "host_problems.cpp", "host_plan.cpp", "host_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in ordinary VGPRs: without this the allocator
         # keeps loop-carried accumulators in VGPRs and copies them to AGPRs
         # around every MFMA chain.
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I" + CSRC, "-I" + INCLUDE, "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "is not a recognized feature" not in l)
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
