"""Builds the CPU oracle (test infrastructure) into oracle/libtfhe_oracle.so.

Plain gcc, no GPU code.  Called by the repository's build entry point and,
when the library is missing, by the oracle's Python wrapper.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtfhe_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "tfhe_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-mavx2", "-ffp-contract=off", "-fPIC", "-shared",
           "-pthread", "-std=c11", "-Wall", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
