"""Build the CPU oracle library (plain C, gcc).

Test infrastructure only.  Compiled with -ffp-contract=off and without
-ffast-math so that every floating-point operation in rto.c is the IEEE
binary64 round-to-nearest operation written in the source; the only fused
multiply-adds are the explicit fma() calls.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librto.so")
SOURCES = [os.path.join(HERE, f) for f in ("rto.c", "dm.c")]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(s) for s in SOURCES + [os.path.join(HERE, "rto.h")])
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", "-o", tmp] + SOURCES + \
          ["-lquadmath", "-lpthread", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
