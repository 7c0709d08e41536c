"""Compile the CPU oracle into oracle/liboracle.so (test infrastructure only).

Flags: no fused multiply-add contraction and no fast-math, so that every fp32
operation is rounded exactly where the source says; OpenMP over pixels.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "msgs_oracle.cpp")
OUT = os.path.join(HERE, "liboracle.so")

FLAGS = ["-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
         "-fPIC", "-shared", "-std=c++17", "-Wall"]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = ["g++", *FLAGS, "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
