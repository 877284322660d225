"""Build the CPU oracle shared library (test infrastructure only).

gcc -O2 -ffp-contract=off keeps every product and sum a separately rounded
IEEE binary64 operation, in source order.  OpenMP is linked for the timed
baseline sweep only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rbf_oracle.c")
LIB = os.path.join(HERE, "librbf_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-missing" not in sys.argv))
