"""Host logic of the request server: the arena free list (compiled with the
host C++ compiler; no GPU)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_arena_free_list():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "arena_check")
        subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_1712_05145_amd", "csrc"),
                        os.path.join(ROOT, "tests", "native", "arena_check.cpp"), "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True)
        assert out.returncode == 0, out.stdout + out.stderr
        assert "OK" in out.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_binding_struct_layout_matches_header():
    """The ctypes structs of the Python binding have the header's layout."""
    import ctypes
    from paper_1712_05145_amd import ffth
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "abi_layout")
        subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "native", "abi_layout.c"), "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        key, val = line.split()
        sname, field = key.split(".")
        cls = getattr(ffth, sname)
        got = ctypes.sizeof(cls) if field == "sizeof" else getattr(cls, field).offset
        assert got == int(val), (key, got, val)
        seen += 1
    assert seen > 20
