"""Build the C oracle (``libwarp_ref.so``) with gcc. Test infrastructure only."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "warp_ref.c")
LIB = os.path.join(HERE, "libwarp_ref.so")

# Baseline x86-64 code: the library is built here and may run on another host.
# -O2, not -O3: gcc 11.4's -O3 loop vectorizer dropped the float32 rounding of
# the displacement (the (double)(float) conversion under the exact-mode test),
# which the mask pins at phase 3/4 catch.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall",
          "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
