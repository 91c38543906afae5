"""Build the CPU oracle library and the host Gray-code timing baseline (test
infrastructure) with gcc."""
from __future__ import annotations

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))

# (source, library, extra flags).  The oracle is built without contraction so
# its canonical sums round as written; the Gray-code baseline is a timing
# reference and is built for speed (its hot loop is cloned for AVX2 and for
# the x86-64 baseline, picked at load time by the CPU it runs on).
_LIBS = [
    ("qubo_oracle.c", "libqubo_oracle.so", ["-O2", "-ffp-contract=off", "-fno-fast-math"]),
    ("gray_cpu.c", "libqubo_gray_cpu.so", ["-O3", "-fno-fast-math"]),
]


def _one(src: str, lib: str, flags: list[str], verbose: bool) -> str:
    out = os.path.join(_HERE, lib)
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", *flags, "-fopenmp", "-fPIC", "-shared", "-o", tmp,
           os.path.join(_HERE, src), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Builds both libraries; returns the oracle's path."""
    outs = [_one(s, l, f, verbose) for s, l, f in _LIBS]
    return outs[0]


def build_gray(verbose: bool = False) -> str:
    s, l, f = _LIBS[1]
    return _one(s, l, f, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
