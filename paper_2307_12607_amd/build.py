"""Build ``libexwarp.so`` (the C-ABI library and its gfx950 kernels) with hipcc, in-tree."""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libexwarp.so")
SOURCES = [os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "warp_forward.hip"),
           os.path.join(CSRC, "warp_backward.hip"), os.path.join(CSRC, "scene_stats.hip"),
           os.path.join(CSRC, "quality.hip"), os.path.join(CSRC, "schedule.cpp"),
           os.path.join(CSRC, "stream_ceiling.hip"), os.path.join(CSRC, "buffer_emd.hip"),
           os.path.join(CSRC, "dynamic_objects.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # The displacement s*u must be rounded once; FMAs are written explicitly.
    "-ffp-contract=off",
    # Keep float32 denormals: tiny displacements must not flush to zero.
    "-fno-gpu-flush-denormals-to-zero",
    # Hardware float32 atomics on coarse-grained device memory.
    "-munsafe-fp-atomics",
    # No packed-FP32 instructions (a hipcc flag; the host pass ignores it).
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-Wno-pass-failed",
]

LINK_FLAGS = ["--offload-arch=gfx950", "-shared", "-fPIC"]


OBJDIR = os.path.join(ROOT, "_build")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source to its own object (in parallel), then link."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 8)
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(lambda src: _compile(src, verbose), SOURCES))
    cmd = [HIPCC, *LINK_FLAGS, *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
