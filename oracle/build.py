"""Build the C oracle (test infrastructure) into oracle/liboracle.so with gcc.

Flags keep IEEE semantics exact: no contraction into fused multiply-add, no
fast-math reassociation, SSE2 binary64 arithmetic (x86-64 default).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")
FLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force=False):
    hdr = os.path.join(HERE, "zig_tables.h")
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(SRC), os.path.getmtime(hdr))
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", *FLAGS, SRC, "-o", tmp, "-pthread", "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
