"""The C ABI from C: tests/c_abi_check.c is compiled as C99 against
include/lbm.h with gcc (warnings are errors), linked to the built library
and run.  It calls host-only entry points, so no GPU is needed."""
import os
import shutil
import subprocess

import pytest

from paper_1703_00185_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_compiles_as_c99_and_library_answers_from_c(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lib = lbm.LIB_PATH
    assert os.path.exists(lib), "build the library first"
    exe = tmp_path / "c_abi_check"
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_check.c"),
           "-o", str(exe), lib, f"-Wl,-rpath,{os.path.dirname(lib)}", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "FAIL" not in run.stdout
