"""Build the HIP library libbbp.so in-tree for gfx950 (hipcc; no JIT cache).

The block-sweep kernels are instantiated per sweep length in separate objects (sweep_kernel.hip compiled
with BBP_KT = 1..6); all objects compile in parallel and are linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbbp.so")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay disabled in every device compile
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

# (source, extra flags, object name)
UNITS = [("plan.cpp", [], "plan.o"), ("bbp.hip", [], "bbp.o"), ("warm.hip", [], "warm.o"),
         ("small_sweep.hip", [], "small_sweep.o"), ("bmps.hip", [], "bmps.o"), ("trunc_sweep.hip", [], "trunc_sweep.o")] + [
    ("sweep_kernel.hip", [f"-DBBP_KT={k}"], f"sweep_k{k}.o") for k in range(1, 7)
]


def _compile(hipcc: str, src: str, extra: list, obj: str, verbose: bool) -> None:
    cmd = [hipcc, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", os.path.join(OBJ, obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src} {' '.join(extra)}")


def build(verbose: bool = True, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, hipcc, src, extra, obj, verbose) for src, extra, obj in UNITS]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *[os.path.join(OBJ, o) for _, _, o in UNITS],
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libbbp.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
