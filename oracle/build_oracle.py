"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle_bdem.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_bdem.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-std=c11",
           "-D_DEFAULT_SOURCE", "-o", LIB + ".tmp", os.path.join(HERE, "bdem_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
