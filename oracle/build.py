"""Build the FP64 CPU oracle shared library (test infrastructure only).

gcc, -O2, -ffp-contract=off so that no multiply-add is fused (neighbour sets
are compared bit-for-bit against the GPU path), OpenMP for the linked-cell
loops.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "md_oracle.c")
LIB = os.path.join(HERE, "_md_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
