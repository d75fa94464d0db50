"""Builds the oracle shared library (plain C, gcc).  Test infrastructure only.

The flags keep IEEE semantics: no fused multiply-add contraction and no
fast-math, so every state operation is a correctly rounded + - * / sqrt.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboxy.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "xy_oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
