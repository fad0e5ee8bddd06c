"""Build the oracle's shared library with gcc (plain C, FP64, no fast-math)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def compile_library(src: str, out: str, verbose: bool = False) -> str:
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-Wall", "-I", HERE, "-o", tmp, src, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    return compile_library(os.path.join(HERE, "oracle.c"), LIB, verbose)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
