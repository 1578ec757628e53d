"""Build libibb.so (HIP for gfx950) next to this file."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "ibb.hip")
HEADERS = [os.path.join(HERE, "csrc", h) for h in ("ivl.hpp", "fam.hpp", "kern.hpp", "tape.hpp", "serve.inc")] + [
    os.path.join(ROOT, "include", "ibb.h")]
LIB = os.path.join(HERE, "libibb.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the interval code relies on IEEE round-up arithmetic: no contraction, no fast-math
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-pthread",
]


def build(force: bool = True, verbose: bool = False) -> str:
    stale = not os.path.exists(LIB) or any(os.path.getmtime(f) > os.path.getmtime(LIB) for f in [SRC, *HEADERS])
    if force or stale:
        tmp = LIB + ".tmp"
        cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, SRC]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
