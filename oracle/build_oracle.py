"""Builds the CPU oracle (plain C, gcc) into oracle/libsblm_oracle.so.

Test infrastructure: the oracle is the reference the HIP library is checked
against.  Compiled without FMA contraction so that every floating-point
operation happens as written (explicit fma() calls are the only fused ones).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["sblm_oracle.c", "ea_oracle.c"]
LIB = os.path.join(HERE, "libsblm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
