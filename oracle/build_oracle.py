"""Compile the FP64 CPU oracle (test infrastructure) into oracle/libdmgs_ref.so.

Plain gcc + OpenMP; no FMA contraction, so every multiply and add is rounded
as written.  Called by the repository's build entry point and, when the
library is missing, by the test fixtures.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dmgs_ref.c")
LIB = os.path.join(HERE, "libdmgs_ref.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
