"""Build the CPU oracle shared libraries (test infrastructure only).

Plain C, double precision, -O2 with FMA contraction off so that every operation is rounded
as written.  The same source is built twice: serial (``libctu_oracle.so``) and with OpenMP
over z-planes (``libctu_oracle_omp.so``); the two give bit-identical results.
Usage: ``python oracle/build.py``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ctu_oracle.c")
LIB = os.path.join(HERE, "libctu_oracle.so")
LIB_OMP = os.path.join(HERE, "libctu_oracle_omp.so")


def build(verbose: bool = False) -> str:
    for lib, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall",
               "-Wextra", "-fPIC", "-shared", *extra, SRC, "-o", lib + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
