"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liblbm_oracle.so.

Plain gcc, -O2, no OpenMP and no fast-math, so the oracle stays the slow,
literal reference it is meant to be.  build(parallel=True) also writes
oracle/liblbm_oracle_omp.so from the same source with -fopenmp, for long
reference runs only (bitwise the same results).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")
LIB_OMP = os.path.join(HERE, "liblbm_oracle_omp.so")


def _compile(out, extra, verbose):
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unknown-pragmas", *extra, "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)


def build(verbose=False, parallel=False):
    _compile(LIB, [], verbose)
    if parallel:
        _compile(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True, parallel=True)
    sys.exit(0)
