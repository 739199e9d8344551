"""Build the C part of the oracle (liboracle_nat.so) with gcc + OpenMP.

Plain -O2 without fast-math flags, so the floating-point order of the C
loops is the order written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_nat.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "nat_ref.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", src,
           "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
