"""Builds the host baseline of the paper's CPU parallel framework
(libfhe_cpupar.so: g++, AVX2, OpenMP; no GPU code)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libfhe_cpupar.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O3", "-mavx2", "-mfma", "-fopenmp", "-std=c++17", "-fPIC", "-shared", "-Wall",
           "-o", tmp, os.path.join(HERE, "cpu_parallel.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
