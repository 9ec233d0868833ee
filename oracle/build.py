"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is compiled by the host C++ compiler with contraction of
multiply-adds switched off, so that its rounding is the plain IEEE rounding
of each written operation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbmd_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built():
    if (not os.path.exists(LIB)) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
