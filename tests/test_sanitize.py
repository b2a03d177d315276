"""CPU sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer).

* The C oracle, built with both sanitizers by gcc, runs its own pins in a
  child process with gcc's ASan runtime preloaded.  The Monte Carlo against
  the 6-D grid (P9) and the MDN normalization quadratures take minutes under
  the sanitizers and are left to ILE_SANITIZE_FULL=1.
* The host side of the C ABI (argument checks, layout conversions, the
  samplers' host logic), built by hipcc with the sanitizers on the host code
  only, runs the host ABI tests with clang's ASan runtime preloaded.  The
  device code is untouched; these tests make no GPU call.

A sanitizer report fails the child (UBSan without recovery), and its output
is checked for reports as well.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _child(env_extra, args, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    return r.returncode, out


def test_oracle_pins_under_sanitizers():
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                              text=True).stdout.strip()
    if not os.path.isabs(gcc_asan) or not os.path.exists(gcc_asan):
        pytest.skip("gcc's ASan runtime is not installed")
    from oracle import build
    lib = build.build(sanitize=True)
    pins = ["tests/test_oracle_pins.py", "tests/test_sampler_pins.py",
            "tests/test_prior_density_pins.py", "tests/test_mdn_pins.py",
            "tests/test_harvest_pins.py", "tests/test_qvu_pins.py", "tests/test_rom_pins.py"]
    args = list(pins)
    if os.environ.get("ILE_SANITIZE_FULL") != "1":
        args += ["-k", "not P9 and not conditionals_integrate_to_one"]
    rc, out = _child({"LD_PRELOAD": gcc_asan, "ILE_ORACLE_LIB": lib}, args, timeout=1500)
    assert not any(t in out for t in REPORTS), out[-4000:]
    assert rc == 0, out[-4000:]


def _stale(target, sources):
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(s) > t for s in sources)


def test_host_abi_under_sanitizers():
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc is not installed")
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's ASan runtime is not installed")
    from paper_1902_04934_amd import build
    srcs = [os.path.join(build.HERE, s) for s in build.SOURCES]
    srcs += glob.glob(os.path.join(build.HERE, "csrc", "*.h"))
    srcs += [os.path.join(ROOT, "include", "ile.h")]
    lib = build.LIB_SAN
    if _stale(lib, srcs):
        build.build(sanitize=True)
    rc, out = _child({"LD_PRELOAD": rt[-1], "ILE_LIB": lib},
                     ["tests/test_abi.py", "tests/test_bench_host.py"], timeout=900)
    assert not any(t in out for t in REPORTS), out[-4000:]
    assert rc == 0, out[-4000:]
