"""Compile the plain-C FP64 oracle into oracle/liboracle.so (test infrastructure)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ppcg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
OMP_SRC = os.path.join(HERE, "ppcg_omp.c")
OMP_LIB = os.path.join(HERE, "liboracle_omp.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    # the paper's CPU baseline (PIPECG-OpenMP), a timing build
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", OMP_LIB, OMP_SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer (CPU
    tests only): any out-of-bounds access or undefined operation aborts."""
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
