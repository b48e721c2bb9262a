"""Build the CPU oracle shared library (test infrastructure; g++, FP64, OpenMP)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libzema_ref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "zema_ref.cpp")
    # -O3 for the timed CPU baseline; no fused multiply-add, so the arithmetic is the
    # source's order (portable x86-64 code: the library may run on another host)
    cmd = ["g++", "-O3", "-ffp-contract=off", "-std=c++17", "-fopenmp", "-fno-fast-math", "-shared", "-fPIC",
           "-Wall", "-o", LIB + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
