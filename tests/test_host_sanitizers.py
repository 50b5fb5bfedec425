"""The oracle and the library's host-only code (keys, encryption, key files,
circuit builders and level schedules) built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc / g++, CPU only) and driven through their
entry points: any out-of-bounds access, leak or undefined behaviour aborts
the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off"]


def build_and_run(tmp_path, compiler, std, sources, libs, args=()):
    exe = str(tmp_path / "driver")
    cmd = [compiler, f"-std={std}", *SAN, f"-I{os.path.join(ROOT, 'include')}", *sources, "-o", exe, *libs]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, cwd=str(tmp_path), timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2005_01945_amd", "csrc")
    out = build_and_run(tmp_path, "g++", "c++17",
                        [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                         os.path.join(csrc, "host_crypto.cpp"), os.path.join(csrc, "circuit_build.cpp")],
                        ["-lpthread"], [str(tmp_path / "keys.bin")])
    assert "host checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "gcc", "c11",
                        [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                         os.path.join(ROOT, "oracle", "tfhe_oracle.c")],
                        ["-pthread", "-lm"])
    assert "oracle checks passed" in out
