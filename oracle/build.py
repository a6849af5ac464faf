"""Build the oracle's plain C routines (gcc, OpenMP).  Test infrastructure."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "knn_fp64.c")
    out = os.path.join(HERE, "libknn_fp64.so")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
