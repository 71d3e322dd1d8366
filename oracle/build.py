"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C compiled with gcc at -O2.  Loop-idiom replacement is
switched off so that its byte loops stay byte loops (the oracle is meant to be
the literal definition, not a tuned copy routine).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hicr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c11", "-O2", "-fno-tree-loop-distribute-patterns",
        "-fPIC", "-shared", "-Wall", "-Wextra", "-Werror",
        "-o", LIB + ".tmp", SRC,
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
