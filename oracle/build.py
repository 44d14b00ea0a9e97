"""Compile the C oracle into ``oracle/libkboracle.so`` (plain gcc, no GPU code)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kb_oracle.c")
LIB = os.path.join(HERE, "libkboracle.so")


# all-cores timing harness: the oracle linked with an OpenMP driver of its element routine
PAR_SRC = os.path.join(HERE, "timing_par.c")
PAR_LIB = os.path.join(HERE, "libkboracle_par.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    par = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", PAR_LIB + ".tmp", SRC, PAR_SRC, "-lm"]
    for c, out in ((cmd, LIB), (par, PAR_LIB)):
        if verbose:
            print(" ".join(c), flush=True)
        subprocess.run(c, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
