"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build.py

compiles ``lbm_oracle.c`` with gcc into ``liblbm_oracle.so`` next to it.
No ``-march`` flag is given, so no fused multiply-add is generated on x86-64
and every product and sum is rounded separately.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
