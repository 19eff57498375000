"""Build the C oracle into shared libraries (test infrastructure only).

Two libraries are built from the same source: ``liboracle.so`` in IEEE
double and ``liboracle_ld.so`` in x87 extended precision (a brute-force
reference for the double one).  Flags: no floating-point contraction other
than the explicit fma calls, OpenMP for the round-robin and many-problem
entry points.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jsvd_oracle.c")
OUT_DIR = os.path.join(HERE, "_lib")
LIBS = {
    "double": os.path.join(OUT_DIR, "liboracle.so"),
    "extended": os.path.join(OUT_DIR, "liboracle_ld.so"),
}
CFLAGS = ["-O2", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    for prec, out in LIBS.items():
        cmd = ["gcc", *CFLAGS, SRC, "-o", out + ".tmp", "-lm"]
        if prec == "extended":
            cmd.insert(1, "-DORACLE_LONG_DOUBLE")
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIBS


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
