"""Build the oracle's shared library (plain C, gcc, no fast-math).

Test infrastructure: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use the oracle.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhsgref.so")
SRC = os.path.join(HERE, "hsgref.c")


def build(force=True):
    """Compile oracle/hsgref.c into oracle/libhsgref.so."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wno-unknown-pragmas", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
