"""Compile the oracle's plain C pair sums (test infrastructure only).

Builds ``oracle/liboracle_p2p.so`` from ``oracle/p2p_ref.c`` with gcc and
OpenMP.  Nothing in the GPU library links this file.

``native=True`` builds the same source with ``-O3 -march=native`` into
``liboracle_p2p_native.so``.  It serves only the hours-long runs that write
stored reference solutions (``tests/golden/make_golden.py``), and is loaded
when ``MFS_ORACLE_NATIVE=1``: the arithmetic is the same loops, with the
compiler free to fuse multiply-adds (rounding differences at the 1e-16
level).  Tests and the CPU baseline use the default build."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "p2p_ref.c")
LIB = os.path.join(HERE, "liboracle_p2p.so")
LIB_NATIVE = os.path.join(HERE, "liboracle_p2p_native.so")


def build(force: bool = True, native: bool = False) -> str:
    lib = LIB_NATIVE if native else LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    tmp = lib + f".tmp{os.getpid()}"
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", *opt, "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(force=True, native="--native" in sys.argv))
    sys.exit(0)
