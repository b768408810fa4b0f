"""Build the C part of the oracle (test infrastructure) into oracle/liborc.so.

    python oracle/build.py

gcc with -O2 -fno-fast-math -ffp-contract=off: every product and sum is rounded
on its own, in source order.  The oracle is single-threaded on purpose: it is
the serial CPU baseline.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c99",
           "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
