"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): a copy of the library is built with the sanitizers applied to the
host pass only (device code is built as usual), and the C client
tests/c_abi_check.c, built with the same compiler and sanitizers, drives the
host-only entry points through it: configuration validation and layout
sizes, model tables and wall factors, error strings, and the argument checks
of every entry point."""
import os
import shutil
import subprocess

import pytest

from paper_1703_00185_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
SANITIZERS = "address,undefined"


@pytest.mark.timeout(900)
def test_host_code_clean_under_address_and_ub_sanitizers(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("ROCm clang not found")
    try:
        build.hipcc()
    except RuntimeError:
        pytest.skip("no HIP compiler")
    lib = str(tmp_path / "libd2q37_san.so")
    host_only = ["-Xarch_host", f"-fsanitize={SANITIZERS}",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]
    build.build(extra_flags=host_only, out=lib)
    exe = str(tmp_path / "c_abi_check_san")
    subprocess.run([CLANG, "-std=c99", "-Wall", "-Werror", f"-fsanitize={SANITIZERS}",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_check.c"),
                    "-o", exe, lib, f"-Wl,-rpath,{tmp_path}", "-lm"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ,
               # the HIP runtime keeps process-lifetime allocations
               ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "FAIL" not in run.stdout
    assert "AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
