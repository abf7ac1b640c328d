"""Host logic compiled with the host C++ compiler (no GPU): the request
server's arena free list and admission order, the descriptor checks of
binary16 launches, and the ctypes struct layouts against the C header."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run_native(src, extra, tag):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, tag)
        subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror"] + extra +
                       ["-I", os.path.join(ROOT, "paper_1712_05145_amd", "csrc"),
                        os.path.join(ROOT, "tests", "native", src), "-o", exe], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        out = subprocess.run([exe], capture_output=True, text=True, env=env)
        assert out.returncode == 0, out.stdout + out.stderr
        assert "OK" in out.stdout
        assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr


# arena free list, admission order of the request server, descriptor checks
# before binary16 launches; each built plain and under AddressSanitizer +
# UndefinedBehaviorSanitizer
NATIVE = ["arena_check.cpp", "admission_check.cpp", "desc_check.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
@pytest.mark.parametrize("src", NATIVE)
@pytest.mark.parametrize("sanitize", [False, True])
def test_host_bookkeeping(src, sanitize):
    _run_native(src, SANITIZE if sanitize else [], src.split(".")[0] + ("_san" if sanitize else ""))


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
