"""Compile the C oracle into oracle/_build/liboracle.so with gcc.

FP64, no fast-math, no floating-point contraction; OpenMP splits independent
zones between threads and never changes the arithmetic of a zone.

build() makes the portable library the tests load (generic x86-64 code, so
that a library built on one host runs on another).  build(native=True) makes
liboracle_native.so with -march=native for timing the oracle on the host that
runs it; with contraction off and no fast-math, both give the same bits.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fargo_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")
LIB_NATIVE = os.path.join(OUT_DIR, "liboracle_native.so")

FLAGS = ["-std=gnu11", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas"]


def build(verbose: bool = False, native: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    out = LIB_NATIVE if native else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + FLAGS + (["-march=native"] if native else []) + [SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True, native="--native" in sys.argv)
    sys.exit(0)
