"""Build the CPU oracle library (plain C, FP64, OpenMP, no fast-math).

TEST INFRASTRUCTURE ONLY: the library built here is loaded by the tests, the
smoke check and the CPU-baseline leg of the benchmark, never by the GPU path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hwenou_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False, out=None, plant=0):
    """Compile the oracle into `out` (default: oracle/liboracle.so).  `plant`
    selects one of the known mistakes of the ORACLE_PLANT switch; the tests
    build such variants elsewhere to show that the pins fail on them."""
    lib = out or LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", f"-DORACLE_PLANT={int(plant)}",
           SRC, "-o", lib + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
