"""Compile the CPU oracle (plain C, gcc) into ``oracle/liboracle.so``.

Test infrastructure only: the product library never links or loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "alias_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# -ffp-contract=off: the double-double routines rely on every + and * being a
# separately rounded IEEE operation; fma() is called explicitly where wanted.
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
          "-shared", "-fPIC"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
