"""Build the WENO-ZA6 oracle (test infrastructure) into oracle/liboracle_za.so.

The oracle is plain C++ compiled with -O2 -ffp-contract=off so every product
and sum is rounded separately, exactly as written.  OpenMP only splits rows
across threads; each interface flux is computed independently and the only
reductions are maxima, so the thread count never changes a result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "za_oracle.cpp")
LIB = os.path.join(HERE, "liboracle_za.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp",
           "-std=c++17", SRC, "-lquadmath", "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
