"""The C ABI from plain C (CPU only): tests/c_client/fk_client.c, a C11
program that includes include/fk.h and links libfkmi.so with no Python or
C++ in between, compiles warning-free and loads the library; run without
arguments it prints its usage and exits 1 before any HIP call."""
import os
import shutil
import subprocess
import sys

import pytest

import paper_2508_07071_amd as fk

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "c_client"))
import build_client  # noqa: E402


def test_c_client_builds_and_loads_the_library():
    if not shutil.which("gcc") or not os.path.exists(fk.LIB_PATH):
        pytest.skip("gcc or libfkmi.so missing")
    exe = build_client.build()  # in-tree: its run path is relative to its folder
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr, (r.returncode, r.stderr)
    ldd = subprocess.run(["ldd", exe], capture_output=True, text=True).stdout
    assert "libfkmi.so" in ldd and "not found" not in ldd, ldd
