"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc.

FP64, -O2 and -ffp-contract=off: the troubled-cell discriminant must be evaluated without fused
multiply-adds so that its decisions match the GPU's bit for bit.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "hgks_oracle.c")
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-D_GNU_SOURCE", "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized",
           src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
