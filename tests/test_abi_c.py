"""The C ABI used from a C program (tests/c_api/abi_check.c): include/mlc.h
compiles as strict C99 and the program, linked against libmlc.so, runs the
host-only checks (problem validation and sizing, status strings, error
paths that need no device)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1702_08111_amd")


def test_c_program(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    assert os.path.exists(os.path.join(PKG, "libmlc.so")), "libmlc.so is not built"
    exe = tmp_path / "abi_check"
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_api", "abi_check.c"), "-o", str(exe),
           "-L", PKG, "-l:libmlc.so", "-Wl,-rpath," + PKG]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
