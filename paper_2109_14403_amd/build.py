"""Build libhom.so (HIP, gfx950) in-tree.

Each pipeline length is its own translation unit (pipe_inst.hip compiled with
-DHOM_N=<n>) so the kernels compile in parallel; everything links into
``paper_2109_14403_amd/libhom.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhom.so")
LENGTHS = (16, 24, 32, 48, 64, 96, 128, 256)
ARCH = os.environ.get("HOM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wno-unused-value",
    "-Wno-unused-command-line-argument",
    # packed FP32 instructions are left to the compiler's scalar code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return p


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    units = []
    for n in LENGTHS:
        units.append((os.path.join(CSRC, "pipe_inst.hip"), os.path.join(BUILD, f"pipe_{n}.o"), [f"-DHOM_N={n}"]))
    for name in ("pointwise", "runtime", "mlp", "dmn", "surrogate", "api"):
        units.append((os.path.join(CSRC, f"{name}.hip"), os.path.join(BUILD, f"{name}.o"), []))

    def compile_one(u):
        src, obj, extra = u
        cmd = [hipcc] + FLAGS + extra + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)
        return obj

    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, units))
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
