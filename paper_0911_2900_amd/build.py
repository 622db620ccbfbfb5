"""Builds libfast.so (HIP for gfx950) in the package directory with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfast.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = os.environ.get("CLANGXX", "/opt/rocm/llvm/bin/clang++")   # host-only C++ sources
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
          f"-I{os.path.join(HERE, '..', 'include')}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = ["plan_batch.hip", "plan_one.hip", "motion.hip", "stream.hip", "cus.hip", "regions.hip", "scratch.hip", "trail.hip",
           "builder.cpp",
           "runtime.cpp"]
# plan_fixed.hip and plan_het.hip are compiled once per v_max (PLAN_V), into
# one object each.
PER_V = ("plan_fixed.hip", "plan_het.hip")
V_MAX = 5


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def _compile_cmd(src: str, v: int = 0):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + (f".v{v}" if v else "") + ".o")
    if src.endswith(".hip"):
        defs = [f"-DPLAN_V={v}"] if v else []
        cmd = [HIPCC, "-x", "hip", *DEVICE, *COMMON, *defs, "-c", path, "-o", obj]
    else:
        cmd = [CLANGXX, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON,
               "-c", path, "-o", obj]
    return cmd, obj


def build(verbose: bool = False) -> str:
    """Compiles every source (always, in parallel) and links
    paper_0911_2900_amd/libfast.so."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(BUILD, exist_ok=True)
    jobs = [_compile_cmd(src, v) for src in PER_V for v in range(V_MAX, 0, -1)]
    jobs += [_compile_cmd(src) for src in SOURCES]
    if verbose:
        for cmd, _ in jobs:
            print(" ".join(cmd), flush=True)
    workers = max(1, min(len(jobs), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        list(pool.map(lambda j: _run(j[0]), jobs))
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
