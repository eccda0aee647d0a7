"""Build the FP64 CPU oracle shared library (test infrastructure only).

    python oracle/build.py

writes oracle/libkbc_oracle.so.  Flags keep IEEE semantics: no fast-math and
no floating-point contraction, so every product and sum rounds once.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["kbc_oracle.c", "kbc_oracle_adj.c"]
OUT = os.path.join(HERE, "libkbc_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
          "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, *[os.path.join(HERE, s) for s in SOURCES], "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
