"""The CPU test suite under AddressSanitizer and UndefinedBehaviorSanitizer.

    python tests/sanitize_cpu.py [extra pytest arguments]

Builds, into paper_2310_19373_amd/_build/san/, instrumented copies of the
host code -- the C oracle, the host Gray-code baseline and the host side of
the HIP library (argument validation, workspace layout, tuning; its device
code is compiled as usual, uninstrumented) -- with LLVM's clang, so that all
three share one sanitizer runtime, and runs ``pytest -m "not gpu"`` against
them with that runtime preloaded into Python.  For the CPU container only:
no GPU is touched (the GPU tests are deselected).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2310_19373_amd")
OUT = os.path.join(PKG, "_build", "san")
LLVM = "/opt/rocm/llvm/bin"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan"]
HOST_SAN = [f for x in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                        "-shared-libsan") for f in ("-Xarch_host", x)]


def run(cmd, **kw):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, **kw)


def build():
    os.makedirs(OUT, exist_ok=True)
    c_flags = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fPIC", "-shared", *SAN]
    run([f"{LLVM}/clang", *c_flags, "-ffp-contract=off", "-o", f"{OUT}/libqubo_oracle.so",
         os.path.join(ROOT, "oracle", "qubo_oracle.c"), "-lm"])
    run([f"{LLVM}/clang", *c_flags, "-o", f"{OUT}/libqubo_gray_cpu.so",
         os.path.join(ROOT, "oracle", "gray_cpu.c"), "-lm"])
    sys.path.insert(0, ROOT)
    from paper_2310_19373_amd import build as lib_build

    objs = []
    for src in sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip"))):
        obj = os.path.join(OUT, os.path.basename(src)[:-4] + ".o")
        run([lib_build.HIPCC, *lib_build.FLAGS, "-g", *HOST_SAN, "-c", src, "-o", obj])
        objs.append(obj)
    run([f"{LLVM}/clang++", "-shared", *SAN, "-o", f"{OUT}/libqubo_bf.so", *objs, "-L/opt/rocm/lib",
         "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])


def runtime():
    out = subprocess.check_output([f"{LLVM}/clang", "-print-file-name=libclang_rt.asan-x86_64.so"], text=True)
    path = out.strip()
    if not os.path.isabs(path):
        path = glob.glob(f"/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")[0]
    return path


def main():
    build()
    env = dict(os.environ)
    env.update({
        "QUBO_ORACLE_LIB": f"{OUT}/libqubo_oracle.so",
        "QUBO_GRAY_LIB": f"{OUT}/libqubo_gray_cpu.so",
        "QUBO_BF_LIB": f"{OUT}/libqubo_bf.so",
        "LD_PRELOAD": runtime(),
        # Python itself is not instrumented: its allocations are not leaks of ours
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-x", "-m", "not gpu",
           "-p", "no:cacheprovider", *sys.argv[1:]]
    print(" ".join(cmd), flush=True)
    sys.exit(subprocess.call(cmd, env=env, cwd=ROOT))


if __name__ == "__main__":
    main()
