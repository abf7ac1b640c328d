"""Build libffth.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1712_05145_amd.build

Compiles the FFT-pass kernels once per precision, the common kernels and the
host driver in parallel, then links the shared library next to this file.
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libffth.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions (v_pk_*_f32) in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]

UNITS = [
    ("ffth_kernels_fft.hip", "k_fft_f32.o", ["-DFFTH_REAL=float"]),
    ("ffth_kernels_fft.hip", "k_fft_f64.o", ["-DFFTH_REAL=double"]),
    ("ffth_kernels_common.hip", "k_common.o", []),
    ("ffth_kernels_multi.hip", "k_multi.o", []),
    ("ffth_host.hip", "host.o", []),
    ("ffth_noalloc.hip", "noalloc.o", []),
]


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    t0 = time.time()
    procs = []
    for src, obj, extra in UNITS:
        cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed = True
            sys.stderr.write("FAILED: " + " ".join(cmd) + "\n" + "\n".join(lines) + "\n")
        elif lines and verbose:
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("hipcc compilation failed")
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + \
        [os.path.join(BUILD, u[1]) for u in UNITS]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build()
