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
