"""Host logic of bench.py: the algorithmic byte model behind the roofline and
the gate that reports measured HBM traffic only for the kernel sources the
counters were taken on.  CPU only."""
import os
import shutil

import pytest

import bench

# Field sizes per voxel and load (the half spectrum holds n/2 of n complex
# values per component, so a spectrum is as large as the real field).
COMP = 6
F32 = COMP * 4            # one FP32 6-component field (or FP32 half spectrum)
H16 = COMP * 2            # binary16 half spectrum
IDS = 2                   # uint16 phase id


def test_inner_iteration_byte_model_from_its_streams():
    m16 = bench.alg_bytes_per_voxel(True)
    m32 = bench.alg_bytes_per_voxel(False)
    # forward y-pass: binary16 spectrum read and written (FP32 without it)
    assert m16["yf"] == H16 + H16 and m32["yf"] == F32 + F32
    # inverse y-pass: FP32 spectrum read and written in both cases
    assert m16["yi"] == m32["yi"] == F32 + F32
    # z-pass: binary16 in, FP32 copy out (FP32 in place without it)
    assert m16["z"] == H16 + F32 and m32["z"] == F32 + F32
    # fused CG pass: FP32 spectrum, r_k, r_k-1, ids read; r_k+1 and the next
    # forward spectrum written; the x pair (two reads, two writes) on every
    # other iteration
    base = F32 + 2 * F32 + IDS + F32
    xpair = (2 * F32 + 2 * F32) / 2
    assert m16["xcg3"] == base + H16 + xpair
    assert m32["xcg3"] == base + F32 + xpair
    # start pass: r_0 and ids read, forward spectrum written
    assert m16["start"] == F32 + IDS + H16 and m32["start"] == F32 + IDS + F32
    # per started solve: no r_k-1 in the first iteration, at most one x pair
    # (read and written) less than the average
    assert bench.XCG3_START_SAVING == F32 + 4 * F32
    # one inner iteration of a load: four passes
    assert m16["xcg3"] + m16["yf"] + m16["z"] + m16["yi"] == 266.0


F64 = COMP * 8            # one FP64 6-component field (or FP64 half spectrum)


def test_fp64_byte_models_count_every_pass():
    """FP64 paths: each application moves the spectrum through two y-passes and
    one z-pass; the order-1 right-hand side adds seven applications per step
    (six displacement transforms and theta); the three-term CG's fused pass
    reads the spectrum, two residuals and ids and writes one residual and the
    spectrum, and moves the x pair on every other iteration."""
    nvox = 1000
    res = [[{"iters": 10, "fp64_applications": 11, "projections": 0}] * 7]
    m = bench.fp64_models(res, nvox, "cg3")
    apps = 7 * 11 + 7
    assert m["ypass_f64"] == nvox * apps * 2 * (F64 + F64)
    assert m["zpass_f64"] == nvox * apps * (F64 + F64)
    assert bench.BYTES["cg3_64"] == F64 + 2 * F64 + IDS + F64 + F64 + (4 * F64) / 2
    assert m["xcg3_f64"] == nvox * (7 * 10 * bench.BYTES["cg3_64"] - 7 * 5 * F64)
    mm = bench.mixed_fp64_models([[{"iters": 60, "fp64_applications": 4, "projections": 2}] * 7], nvox)
    assert mm["ypass_f64"] == nvox * (7 * 4 + 7) * 2 * (F64 + F64)
    # projection: x-forward reads the FP64 residual and ids, writes the FP32 spectrum
    assert mm["xfwd_f32"] == nvox * 14 * (F64 + IDS + F32)


def _copy_tree(dst):
    root = bench.ROOT
    shutil.copytree(os.path.join(root, "paper_1712_05145_amd", "csrc"),
                    os.path.join(dst, "paper_1712_05145_amd", "csrc"))
    shutil.copytree(os.path.join(root, "profiles"), os.path.join(dst, "profiles"))


def test_traffic_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    if bench.measured_traffic("xcg3_f32") is None:
        pytest.skip("kernel sources changed since the counter summary was taken")
    _copy_tree(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    value = bench.measured_traffic("xcg3_f32")
    assert value is not None and value > 0
    # any change to a kernel source voids the recorded traffic
    src = os.path.join(str(tmp_path), "paper_1712_05145_amd", "csrc", "ffth_kernels.h")
    with open(src, "a") as f:
        f.write("\n")
    assert bench.measured_traffic("xcg3_f32") is None
    # and without the summary there is nothing to report
    os.remove(os.path.join(str(tmp_path), "profiles", "traffic_fp32_passes_voronoi256.md"))
    assert bench.measured_traffic("xcg3_f32") is None
