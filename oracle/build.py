"""Compile the CPU oracle (test infrastructure) with gcc: oracle/liboracle.so (serial) and,
from the same source with OpenMP, oracle/liboracle_omp.so (level-parallel entry points)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sta_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-msse2", "-mfpmath=sse", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        cmd = ["gcc", *CFLAGS, *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
