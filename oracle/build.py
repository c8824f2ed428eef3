"""Compile the oracle (plain C, FP64, OpenMP) into oracle/libehd_oracle.so.

Test infrastructure: the product library never links or loads it."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ehd_oracle.c")
LIB = os.path.join(HERE, "libehd_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
