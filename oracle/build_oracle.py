"""Builds the CPU oracle (test infrastructure) with g++: FP64, OpenMP, no
contraction and no fast-math, so the FP32 opening test is evaluated exactly
as written."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle.cpp", "oracle_mac.cpp"]
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src_dir: str = HERE, out: str = OUT) -> str:
    """Compiles the sources in src_dir (default: this folder) into out."""
    srcs = [os.path.join(src_dir, s) for s in SOURCES if os.path.exists(os.path.join(src_dir, s))]
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", out + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
