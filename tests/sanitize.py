#!/usr/bin/env python3
"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the CPU-side code.

Builds, into _build/sanitize/ (ignored by git),
  * the FP64 oracle (gcc, -fsanitize=address,undefined), and
  * libt2s2.so with its host code instrumented (hipcc, -Xarch_host before
    each -fsanitize=; the gfx950 device code is built as usual),
then runs, each in a process of its own with the matching runtime preloaded
and every report fatal:
  * the C-ABI checks that need no GPU (test_abi_cpu.py, test_host_logic.py)
    against the instrumented library, and
  * the oracle's pins (test_oracle_pins.py, test_family_pins.py,
    test_twin_pins.py), without the long paper-table runs, against the
    instrumented oracle.
Exit status 0 when both pass.  Usage: python tests/sanitize.py
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_12913_amd", "csrc")
HIP_SOURCES = ["t2s2_kernels.hip", "t2s2_adjoint.hip", "t2s2_stability.hip", "t2s2_probe.hip",
               "t2s2_api.hip"]
SLOW = ("table_1 or table_2 or table_4 or second_order or t1s2_unstable or "
        "poiseuille_converges or temporal_order")


def run(cmd, env=None):
    print("+ " + " ".join(cmd), flush=True)
    return subprocess.call(cmd, env=env, cwd=ROOT)


def main():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = os.path.join(ROOT, "_build", "sanitize")
    os.makedirs(tmp, exist_ok=True)
    olib = os.path.join(tmp, "liboracle_asan.so")
    hlib = os.path.join(tmp, "libt2s2_asan.so")
    rc = run(["gcc", "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
              "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-o", olib,
              os.path.join(ROOT, "oracle", "t2s2_oracle.c"), "-lm"])
    if rc:
        return rc
    rc = run([os.path.join(rocm, "bin", "hipcc"), "--offload-arch=gfx950", "-O1", "-g",
              "-std=c++17", "-fPIC", "-shared", "-shared-libsan",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
              "-o", hlib] + [os.path.join(CSRC, s) for s in HIP_SOURCES])
    if rc:
        return rc
    common = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                  UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONMALLOC="malloc")
    clang_rt = subprocess.check_output(
        [os.path.join(rocm, "llvm", "bin", "clang"), "-print-file-name=libclang_rt.asan-x86_64.so"],
        text=True).strip()
    if not os.path.exists(clang_rt):
        import glob

        found = glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                       "libclang_rt.asan-x86_64.so"))
        clang_rt = found[0]
    env = dict(common, LD_PRELOAD=clang_rt, T2S2_TEST_LIB=hlib)
    rc_abi = run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                  "tests/test_abi_cpu.py", "tests/test_host_logic.py"], env=env)
    gcc_rt = [subprocess.check_output(["gcc", "-print-file-name=" + n], text=True).strip()
              for n in ("libasan.so", "libubsan.so")]
    env = dict(common, LD_PRELOAD=":".join(gcc_rt), T2S2_TEST_ORACLE_LIB=olib)
    rc_oracle = run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                     "tests/test_oracle_pins.py", "tests/test_family_pins.py",
                     "tests/test_twin_pins.py", "-k", f"not ({SLOW})"], env=env)
    print(f"sanitized C-ABI checks: {'ok' if rc_abi == 0 else 'FAILED'}; "
          f"sanitized oracle pins: {'ok' if rc_oracle == 0 else 'FAILED'}", flush=True)
    return 1 if (rc_abi or rc_oracle) else 0


if __name__ == "__main__":
    sys.exit(main())
