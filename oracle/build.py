"""Build the C oracle (test infrastructure) into oracle/libile_oracle.so.

Plain gcc, -O2, no fast-math and no FMA contraction, OpenMP over samples.
build(sanitize=True) writes oracle/libile_oracle_san.so instead, with
AddressSanitizer and UndefinedBehaviorSanitizer (CPU only; loaded through
ILE_ORACLE_LIB with the ASan runtime preloaded, see tests/test_sanitize.py).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libile_oracle.so")
LIB_SAN = os.path.join(HERE, "libile_oracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    srcs = [os.path.join(HERE, f) for f in ("ile_oracle.c", "mdn_oracle.c")]
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", *(SAN_FLAGS if sanitize else []), "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
