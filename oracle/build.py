"""Build the oracle shared library (plain C, gcc, IEEE double, no contraction;
OpenMP for the optional multi-threaded sweeps, one thread by default).

Test infrastructure only: the HIP library never links or loads this.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smre_oracle.c")
LIB = os.path.join(HERE, "libsmre_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
           "-shared", "-fopenmp", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
