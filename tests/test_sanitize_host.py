"""The oracle and libsta's host code built with AddressSanitizer and UndefinedBehavior-
Sanitizer (gcc/g++, CPU only) and driven over seeded designs and planted bad inputs in a
child process; any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return os.path.realpath(p) if p and os.path.isabs(p) and os.path.exists(p) else None


def test_sanitized_host_code_and_oracle(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    orc = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
                           "-o", str(orc), os.path.join(ROOT, "oracle", "sta_oracle.c"), "-lm"])
    host = tmp_path / "libsta_host_san.so"
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                           "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-w",
                           "-o", str(host), os.path.join(ROOT, "paper_2203_08395_amd", "csrc", "sta_graph.cpp"),
                           os.path.join(ROOT, "tests", "sanitize", "host_stubs.cpp")])
    env = dict(os.environ, LD_PRELOAD=f"{asan} {ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize", "driver.py"), str(orc), str(host),
                        ROOT], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "clean" in r.stdout
