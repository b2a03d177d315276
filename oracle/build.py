"""Build the C oracle (test infrastructure) into oracle/libile_oracle.so.

Plain gcc, -O2, no fast-math and no FMA contraction, OpenMP over samples.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libile_oracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, f) for f in ("ile_oracle.c", "mdn_oracle.c")]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
