"""Build libile.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libile.so")
SOURCES = ["csrc/ile_kernels.hip", "csrc/ile_sampler.hip", "csrc/ile_batch.hip",
           "csrc/ile_mdn.hip", "csrc/ile_harvest.hip", "csrc/ile_qvu.hip", "csrc/ile_rom.hip",
           "csrc/ile_api.cpp", "csrc/ile_batch_api.cpp", "csrc/ile_prop_api.cpp"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every HIP kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"),
               "-I", os.path.join(HERE, "csrc"), "-c", os.path.join(HERE, src),
               "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip", *HIP_FLAGS, "-I", os.path.join(ROOT, "include"),
                   "-I", os.path.join(HERE, "csrc"), "-c", os.path.join(HERE, src),
                   "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
