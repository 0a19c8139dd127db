"""Compile the CPU oracle (test infrastructure) into oracle/libocfd_oracle.so.

The flags keep the arithmetic literal: no contraction into fused multiply-adds
and no value-changing optimisations, so the oracle evaluates each formula as
written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ocfd_oracle.c")
LIB = os.path.join(HERE, "libocfd_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
