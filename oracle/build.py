"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/liboracle.so``.

The oracle is compiled with plain g++, no FMA contraction and no fast-math, so
its arithmetic is exactly the op order written in ``oracle.cpp``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

CXXFLAGS = ["-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
            "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    """Compile ``oracle.cpp``; returns the library path.  Raises on failure."""
    tmp = LIB + ".tmp"
    cmd = ["g++", *CXXFLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
