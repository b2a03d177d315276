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


# host-side sanitizers only (the device code is built as usual)
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host",
            "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
LIB_SAN = os.path.join(HERE, "libile_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link libile.so.  sanitize=True
    writes libile_san.so instead, its host code (argument checks, layout
    conversions, the samplers' host logic) built with AddressSanitizer and
    UBSan; it runs with the clang ASan runtime preloaded."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    bdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    os.makedirs(bdir, exist_ok=True)
    flags = HIP_FLAGS + (HOST_SAN if sanitize else [])
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *flags, "-I", os.path.join(ROOT, "include"),
               "-I", os.path.join(HERE, "csrc"), "-c", os.path.join(HERE, src),
               "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip", *flags, "-I", os.path.join(ROOT, "include"),
                   "-I", os.path.join(HERE, "csrc"), "-c", os.path.join(HERE, src),
                   "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-shared-libsan"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
