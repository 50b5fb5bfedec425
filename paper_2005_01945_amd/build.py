"""Builds the HIP library libfhe_mi355x.so in-tree (gfx950 device code).

Usage: python -m paper_2005_01945_amd.build [-v] [--resource-usage]
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfhe_mi355x.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["kernels.hip", "runtime.cpp", "host_crypto.cpp", "circuits.cpp", "circuit_build.cpp", "serve.cpp",
           "tuner.cpp", "noalloc.cpp"]
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          # no packed-FP32 instructions anywhere in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # keep host floating point (Box-Muller noise) free of contractions
          "-ffp-contract=off",
          f"-I{os.path.join(ROOT, 'include')}"]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str, verbose: bool, resource_usage: bool) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [_hipcc(), f"--offload-arch={ARCH}", *COMMON, "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    if resource_usage and src.endswith(".hip"):
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 or (verbose and r.stderr):
        sys.stderr.write(r.stderr)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed")
    return obj


def build(verbose: bool = False, resource_usage: bool = False, out: str = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, resource_usage), SOURCES))
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    out = None
    if "-o" in sys.argv:
        out = os.path.abspath(sys.argv[sys.argv.index("-o") + 1])
    print(build(verbose="-v" in sys.argv, resource_usage="--resource-usage" in sys.argv, out=out))
