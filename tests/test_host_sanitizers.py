"""Host code under the address and undefined-behaviour sanitizers: the CPU
oracle (every entry point on small inputs) and the library's host-only
validation and sliced-ELL builder (valid and malformed CSR).  Each driver is
built with the sanitizers and run in a child process; any out-of-bounds
access, use of freed memory, leak or undefined operation fails it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    _build(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", *FLAGS,
            os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_driver.c"),
            "-o", exe, "-lm"])
    _run(exe)


def test_host_validation_under_sanitizers(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not available")
    exe = str(tmp_path / "validate_san")
    _build([CLANG, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
            "-I" + os.path.join(ROOT, "include"),
            "-I" + os.path.join(ROOT, "paper_2505_22631_amd", "csrc"), *FLAGS,
            os.path.join(ROOT, "paper_2505_22631_amd", "csrc", "validate.cpp"),
            os.path.join(SAN, "validate_driver.cpp"), "-L/opt/rocm/lib", "-lamdhip64",
            "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    _run(exe)
