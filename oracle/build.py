"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, -O2, no fast-math and no floating-point contraction, so every
IEEE operation of the oracle is rounded exactly once in the order written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["pperm_oracle.c", "saw_enum.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra",
           *[os.path.join(HERE, s) for s in SOURCES], "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
