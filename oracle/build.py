"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so, and
the same source with OpenMP into oracle/liboracle_omp.so (the multi-core
CPU baseline; its loops share independent iterations among threads and give
the plain build's results bit for bit).

Plain gcc, no fast-math and no floating-point contraction, so every
arithmetic operation in the oracle is the separately rounded IEEE operation
that its source spells out.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "f3r_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(verbose: bool = False, src: str = SRC, out: str = LIB, openmp: bool = False) -> str:
    """Compile `src` (default: the oracle) into `out`.  The pin tests pass a
    copy of the source with a planted mistake and a path of their own.
    With out = LIB (the default call) the OpenMP build is made as well."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-frounding-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-fopenmp" if openmp else "-fno-openmp",
           "-I", HERE, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    if out == LIB and src == SRC and not openmp:
        build(verbose, SRC, LIB_OMP, openmp=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
