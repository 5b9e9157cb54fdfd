"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so.

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


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile `src` (default: the oracle) into `out`.  The pin tests pass a
    copy of the source with a planted mistake and a path of their own."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-frounding-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-I", HERE, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
