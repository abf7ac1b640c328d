"""Benchmark: FFT-based homogenization on one MI355X.

Workload (default): 256^3 periodic Voronoi polycrystal, 200 seeded grains,
grain Lame pairs log-uniform in [1, 50], reference medium at the midpoint.
One step = the six order-0 unit loads (full 6x6 effective stiffness) followed
by the order-1 problem for the gradient load (grad E)_111 = (grad E)_222 = 1,
whose right-hand side is built from the six order-0 correctors; CG with FP32
inner solves and FP64 defect correction to relative residual 1e-8.

Printed value: voxel-iterations per second of the mixed-precision path
(one voxel-iteration = one voxel x one operator application, FP32 inner and
FP64 residual applications both counted).  Also reported: the plain FP64 GPU
path on the same workload at the same tolerance (speedup), p50/p99 step
latency, the dominant kernel against the HBM roofline (HIP events on the
plan's stream over the timed steps), and the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iters/s at 256^3, mixed vs FP64 to 1e-8 residual; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per voxel for one load in one launch of the FP32
# kernel categories whose traffic does not depend on the mode (4-byte words,
# 2-byte phase ids; the half spectrum is 6 x n/2 complex = 24 B per voxel in
# FP32, 12 B in binary16):
#   y-pass / z-pass        spectrum read and written                 24+24
#   fused three-term CG    spectrum, r_k, r_k-1, phase read; r_k+1
#   x-pass                 and the spectrum written; on odd iterations
#                          also the pair x_k-1, x_k-2 read and x_k+1, x_k
#                          written (48 B a voxel on average)        24*3+2+24*2 + 48
#   start pass of a solve  r_0, phase read; spectrum written          24+2+24
# With the binary16 forward spectrum of the inner solve, every write of the
# spectrum before the spectral operator and every read of it up to there is
# 12 B: forward y-pass 12+12, z-pass 12+24, fused pass 24*3+2+24+12 + 48,
# start pass 24+2+12; the inverse y-pass (24+24) and the projection passes
# stay FP32.  The first iteration of a solve reads no r_k-1 (24 B) and the
# second reads no x pair (x_0 = 0); a solve of K iterations moves 48 or 96 B
# per voxel less x traffic than K times the average: the model subtracts
# 24 + 96 for every start (a lower bound on the bytes moved).  A solve that
# ends after an even iteration forms its last x in a separate finish kernel
# (pointwise category).  The FP32 x-forward / x-inverse categories hold the
# projection passes only.
ALG_CATEGORIES = ("ypass_f32", "zpass_f32", "xcg3_f32", "cg3start_f32")
XCG3_START_SAVING = 120.0


def alg_bytes_per_voxel(h16):
    """Bytes per voxel of (forward y, inverse y, z, fused CG pass averaged over
    an even and an odd iteration, start pass) in the inner solve; projection
    passes move 48 B in each y- and z-pass."""
    if h16:
        return {"yf": 24.0, "yi": 48.0, "z": 36.0, "xcg3": 158.0, "start": 38.0}
    return {"yf": 48.0, "yi": 48.0, "z": 48.0, "xcg3": 170.0, "start": 50.0}


# FP64 words are 8 B: a 6-component FP64 field or FP64 half spectrum is 48 B
# per voxel.  Per-voxel bytes of one load through one launch, by pass mode:
F64 = 48.0
F32W = 24.0
IDB = 2.0
BYTES = {
    # one y-pass (an application has two) and the z-pass of an FP64
    # application: spectrum read and written
    "y64": 2 * F64, "z64": 2 * F64,
    # FP64 residual sweep of the defect correction (x-forward, mode LS): the
    # first sweep reads ids and writes the spectrum (the iterate is zero and
    # not read); later sweeps also read the iterate and the FP32 correction
    # and write the iterate back; order 1 also reads the stored
    # right-hand-side polarization
    "sweep0_xf": IDB + F64, "sweep_xf": IDB + F64 + F32W + F64 + F64, "rhs_P": F64,
    # its x-inverse (mode RESID): spectrum and iterate read, residual written
    # (the first sweep reads no iterate and writes an FP32 residual, which
    # goes straight to the inner solve)
    "sweep0_xi": F64 + F32W, "sweep_xi": F64 + F64 + F64,
    # FP32 projection of the FP64 residual: x-forward (C0 : r) reads r (FP64)
    # and ids and writes the spectrum; y/z 48 each; x-inverse reads the
    # spectrum, x and r (FP64) and writes x (FP64) and the FP32 right-hand side
    "proj_xf": IDB + F64 + F32W, "proj_xi": F32W + F64 + F64 + F64 + F32W,
    # plain two-term CG (FP64): x-forward reads r, p, ids, writes p, spectrum;
    # x-inverse reads spectrum, p, x, r, writes x, r
    "cg_xf": F64 + F64 + IDB + F64 + F64, "cg_xi": F64 + 3 * F64 + 2 * F64,
    # its two start applications: b (iterate zero: read, ids; spectrum
    # written; x-inverse: spectrum and x read, x written) and r_0 = b - A b
    # (x-forward the same; x-inverse: spectrum, x read, r written)
    "ls_xf": IDB + F64 + F64, "bs_xi": F64 + F64 + F64, "resid_xi": F64 + F64 + F64,
    # three-term CG in FP64: fused pass (spectrum, r_k, r_k-1, ids read; r_k+1
    # and the spectrum written; the x pair read and written on odd iterations,
    # 2 x 48 B a voxel on average), start pass, and per started solve the
    # lower-bound saving of the model (no r_k-1 in the first iteration, at
    # most one x pair less than the average)
    "cg3_64": F64 + 2 * F64 + IDB + F64 + F64 + 2 * F64, "cg3s_64": F64 + IDB + F64,
    "cg3_64_saving": F64 + 4 * F64,
}


def measured_traffic(cat):
    """HBM bytes per algorithmic byte of kernel category `cat` from the
    committed counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on device
    copies), or None when the kernel sources changed since it was taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1712_05145_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    path = os.path.join(ROOT, "profiles", "traffic_fp32_passes_voronoi256.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    if f"source-hash: {h.hexdigest()[:16]}" not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith(f"traffic-ratio {cat}:"):
            return float(line.split(":")[1])
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def default_grad():
    g = np.zeros((6, 3))
    g[0, 0] = 1.0      # dE_11/dY_1
    g[1, 1] = 1.0      # dE_22/dY_2
    return g.reshape(1, 18)


def _oracle_apply_worker(job):
    """One FP64 operator application of the oracle (child process)."""
    n_sample, grains, seed, k = job
    from threadpoolctl import threadpool_limits

    from oracle import homogenization as H
    from paper_1712_05145_amd import microstructure as M
    phase, lame = M.voronoi_polycrystal(n_sample, grains, seed)
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    x = np.random.default_rng(k).standard_normal((3, 3) + phase.shape)
    x = 0.5 * (x + np.swapaxes(x, 0, 1))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        prob.apply_A(x)
        return time.perf_counter() - t0


def host_info():
    import platform
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "machine": platform.machine()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz")
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keep:
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(n_sample, grains, seed, apps_per_step, n_full, workers):
    """The FP64 oracle on the host cores: `workers` processes each apply the
    oracle's operator once (FFT, Green operator, inverse FFT) to their own field
    on the n_sample^3 Voronoi polycrystal of the same generator, all at once;
    the rate is voxels x applications / wall time.  The time the oracle would
    take for one benchmark step (apps_per_step FP64 applications at n_full^3,
    the iteration count of plain FP64 CG) is extrapolated by N^3 log N."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_oracle_apply_worker, [(n_sample, grains, seed, k) for k in range(workers)])
    wall = time.perf_counter() - t0
    nv = n_sample ** 3
    rate = workers * nv / max(per)
    scale = (n_full ** 3 * np.log(n_full ** 3)) / (nv * np.log(nv))
    # the step's seven solves are independent: at most seven run at once
    par = min(workers, 7)
    step_s = apps_per_step * max(per) * scale / par if apps_per_step else None
    return {"value": round(rate, 1), "unit": "voxel-iters/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} processes, one FP64 operator application each (FFT, Green operator, inverse FFT) "
                      f"of the oracle on the {n_sample}^3 Voronoi polycrystal of the same generator, at once; "
                      f"{max(per):.1f} s per application, {wall:.1f} s wall with process start",
            "grid": n_sample, "seconds_per_application": round(max(per), 2),
            "step_extrapolated_s": None if step_s is None else round(step_s, 1),
            "step_extrapolation": f"{apps_per_step} FP64 applications of the {n_full}^3 step (plain FP64 CG "
                                  f"iteration count) x the sampled time per application x N^3 log N scaling, "
                                  f"spread over {par} processes (one per load case)",
            "host": host_info()}


def spheres128_run(dev):
    """Random-sphere composite at 128^3 (20 non-overlapping spheres, Young
    contrast 100, nu 0.3): the six unit loads with the Basic Scheme and with CG,
    FP32 inner solves under FP64 defect correction to 1e-8."""
    import torch

    from paper_1712_05145_amd import ffth
    from paper_1712_05145_amd import microstructure as M
    phase, lame = M.random_spheres(128, 20, seed=2)
    lam0, mu0 = M.midpoint_reference(lame)
    out, ceffs = {}, {}
    for scheme in ("cg", "basic"):
        s = ffth.Solver(phase, lam0, mu0, lame=lame, nloads=6, scheme=scheme, precision="mixed", tol=1e-8,
                        max_iter=50000, device=dev)
        s.solve_order0(np.eye(6))                        # warm-up (tile tuning, first launches)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, res = s.solve_order0(np.eye(6))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        apps = sum(r["iters"] + r["projections"] + r["fp64_applications"] for r in res)
        out[scheme] = {"ms": round(dt * 1e3, 2), "fp32_inner": sum(r["iters"] for r in res),
                       "fp64_applications": sum(r["fp64_applications"] for r in res),
                       "voxel_iters_per_s": round(phase.size * apps / dt, 1)}
        ceffs[scheme] = np.array([r["mean_stress"] for r in res]).T
        s.close()
    d = np.sqrt(np.outer(np.diag(ceffs["cg"]), np.diag(ceffs["cg"])))
    out["ceff_cg_vs_basic_max_scaled_diff"] = float(np.max(np.abs(ceffs["cg"] - ceffs["basic"]) / d))
    log(f"spheres128: CG {out['cg']['ms']} ms, Basic Scheme {out['basic']['ms']} ms")
    return out


def fp32_only_run(dev, phase, lame, lam0, mu0, eps0_ref, ceff_ref):
    """FP32-only solves (no FP64 defect correction) with their measured error
    against the refined result of the same problem: the 16^3 centred sphere
    (Young contrast 10; Basic Scheme and CG, load e_11), the 128^3 random
    spheres (contrast 100; CG, six unit loads) and the benchmark polycrystal
    (CG, six unit loads, against the mixed step's correctors).  Tolerance 1e-6
    on the recursive residual, at most 3000 iterations: where FP32 stalls above
    it the status says so and the error is still the measured one."""
    import torch

    from paper_1712_05145_amd import ffth
    from paper_1712_05145_amd import microstructure as M
    out = {}

    def one(name, ph, lm, l0, m0, scheme, E, ref_eps, ref_ceff):
        s = ffth.Solver(ph, l0, m0, lame=lm, nloads=len(E), scheme=scheme, precision="fp32", tol=1e-6,
                        max_iter=3000, device=dev)
        eps, res = s.solve_order0(E, check=False)
        s.close()
        e = {"scheme": scheme, "tol": 1e-6, "status": [r["status"] for r in res],
             "iters": [r["iters"] for r in res], "recursive_residual": [r["residual"] for r in res],
             "field_rel_l2": max(field_rel_l2(eps[i:i + 1], ref_eps[i:i + 1]) for i in range(len(E)))}
        if ref_ceff is not None:
            e["ceff_max_scaled_diff"] = ceff_scaled_diff(np.array([r["mean_stress"] for r in res]).T, ref_ceff)
        else:
            e["mean_stress_rel"] = float(np.abs(np.array(res[0]["mean_stress"]) - ref_ceff_vec).max()
                                         / np.abs(ref_ceff_vec).max())
        out[name] = e
        del eps
        torch.cuda.empty_cache()

    # config 1: centred sphere 16^3, load e_11, reference FP64 at 1e-12
    ph1, lm1 = M.centred_sphere(16, young=(1.0, 10.0))
    l1, mu1 = M.midpoint_reference(lm1)
    r1 = ffth.Solver(ph1, l1, mu1, lame=lm1, scheme="basic", precision="fp64", tol=1e-12, device=dev)
    e1ref, rr1 = r1.solve_order0([1, 0, 0, 0, 0, 0])
    r1.close()
    ref_ceff_vec = np.array(rr1[0]["mean_stress"])
    for sch in ("basic", "cg"):
        one(f"sphere16_{sch}", ph1, lm1, l1, mu1, sch, np.eye(6)[:1], e1ref, None)
    # config 2: random spheres 128^3, six loads, reference mixed CG at 1e-10
    ph2, lm2 = M.random_spheres(128, 20, seed=2)
    l2, mu2 = M.midpoint_reference(lm2)
    r2 = ffth.Solver(ph2, l2, mu2, lame=lm2, nloads=6, precision="mixed", tol=1e-10, device=dev)
    e2ref, rr2 = r2.solve_order0(np.eye(6))
    r2.close()
    one("spheres128_cg", ph2, lm2, l2, mu2, "cg", np.eye(6), e2ref, np.array([r["mean_stress"] for r in rr2]).T)
    del e2ref
    # config 3: the benchmark polycrystal
    one("voronoi256_cg", phase, lame, lam0, mu0, "cg", np.eye(6), eps0_ref, ceff_ref)
    log("fp32-only: " + ", ".join(f"{k} {v['field_rel_l2']:.1e}" for k, v in out.items()))
    return out


def fibres_run(dev, n):
    """Aligned fibre composite (70 fibres along x3, radius 0.04, hexagonal
    jittered packing, fibre/matrix Young 1000/1, nu 0.25/0.35) at n^3: the six
    order-0 unit loads and the order-1 load, mixed CG to 1e-8 (the stiffness
    contrast is above the binary16 limit: FP32 inner spectrum).  One step
    after the plans are built and tuned."""
    import torch

    from paper_1712_05145_amd import ffth
    from paper_1712_05145_amd import microstructure as M
    t = time.perf_counter()
    phase, lame = M.hex_fibres(n)
    lam0, mu0 = M.midpoint_reference(lame)
    gen_s = time.perf_counter() - t
    torch.cuda.reset_peak_memory_stats(dev)
    t = time.perf_counter()
    kw = dict(lame=lame, precision="mixed", tol=1e-8, max_iter=50000, device=dev)
    s0 = ffth.Solver(phase, lam0, mu0, nloads=6, **kw)
    s1 = ffth.Solver(phase, lam0, mu0, nloads=1, order=1, **kw)
    plan_s = time.perf_counter() - t
    e0 = s0.field(6, 6)
    e1 = s1.field(6, 1)
    ffth.ffth_profile_enable(s0.plan, True)
    ffth.ffth_profile_enable(s1.plan, True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, r0 = s0.solve_order0(np.eye(6), out=e0)
    _, r1 = s1.solve_order1(e0, default_grad(), out=e1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    prof = merge_prof(ffth.ffth_profile_read(s0.plan), ffth.ffth_profile_read(s1.plan))
    res = r0 + r1
    nvox = phase.size
    inner = sum(r["iters"] for r in res)
    proj = sum(r["projections"] for r in res)
    f64 = sum(r["fp64_applications"] for r in res)
    ab = alg_bytes_per_voxel(False)
    starts = prof["cg3start_f32"][2]
    model = {"xcg3_f32": nvox * (inner * ab["xcg3"] - XCG3_START_SAVING * starts),
             "ypass_f32": nvox * (inner * (ab["yf"] + ab["yi"]) + proj * 96.0),
             "zpass_f32": nvox * (inner * ab["z"] + proj * 48.0), "cg3start_f32": nvox * ab["start"] * starts}
    model.update(mixed_fp64_models([res], nvox))
    ceff = np.array([r["mean_stress"] for r in r0]).T
    out = {"workload": f"fibres{n}-order0x6+order1", "grid": [n] * 3, "stiffness_contrast":
           round(ffth.ffth_stiffness_contrast(lame=lame), 1), "fibre_fraction": round(float(phase.mean()), 4),
           "ms_per_step": round(dt * 1e3, 1), "status": [r["status"] for r in res],
           "fp32_inner": inner, "fp32_projections": proj, "fp64_applications": f64,
           "inner_iters_per_load": [r["iters"] for r in res],
           "voxel_iters_per_s": round(nvox * (inner + proj + f64) / dt, 1),
           "residuals": [r["residual"] for r in res],
           "ceff_diag": [round(float(v), 4) for v in np.diag(ceff)],
           "peak_memory_GB": round(torch.cuda.max_memory_allocated(dev) / 1e9, 1),
           "generation_s": round(gen_s, 1), "plans_s": round(plan_s, 1),
           "kernels": kernel_table(prof, nvox, model)}
    log(f"fibres{n}: {dt * 1e3:.0f} ms, {inner} inner iterations, {f64} FP64 applications, "
        f"peak {out['peak_memory_GB']} GB")
    s0.close()
    s1.close()
    del s0, s1, e0, e1
    torch.cuda.empty_cache()
    return out


def serving_run(count, rate, dev):
    """Request stream: Poisson arrivals, grids 32^3..128^3, random-sphere
    microstructures, six unit loads each, mixed CG to 1e-8, 64 GB arena."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_1712_05145_amd import microstructure as M
    from paper_1712_05145_amd.serving import Server, replay

    stream = M.serving_requests(count=count, rate=rate)

    def gen(r):
        ph, lame = M.overlapping_spheres(r["n"], r["fraction"], r["contrast"], r["seed"])
        return r["id"], (ph, lame) + M.midpoint_reference(lame)

    t = time.perf_counter()
    with ThreadPoolExecutor(8) as ex:
        inputs = dict(ex.map(gen, stream))
    log(f"serving: {count} request microstructures in {time.perf_counter() - t:.1f}s")
    srv = Server(64 << 30, max_running=64, device=dev)
    wid = srv.submit(*inputs[0], np.eye(6))              # warm-up request
    while srv.poll(wid)[0] == 6:
        srv.step()
    records, stats = replay(srv, stream, inputs)
    srv.close()
    offered = sum(r["voxel_iters"] for r in records) / stream[-1]["arrival"]
    by_n = {}
    for n in sorted({r["n"] for r in records}):
        lat = [r["latency"] for r in records if r["n"] == n]
        by_n[str(n)] = {"count": len(lat), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
                        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 1)}
    log(f"serving: p50 {stats['latency_p50_ms']:.0f} ms, p99 {stats['latency_p99_ms']:.0f} ms")
    return {"requests": count, "rate_per_s": rate, "loads_per_request": 6, "makespan_s": round(stats["makespan_s"], 2),
            "latency_p50_ms": round(stats["latency_p50_ms"], 1), "latency_p99_ms": round(stats["latency_p99_ms"], 1),
            "achieved_voxel_iters_per_s": round(stats["voxel_iters_per_s"], 1),
            "offered_voxel_iters_per_s": round(offered, 1), "failed": stats["failed"], "by_grid": by_n,
            "arena_bytes": 64 << 30, "max_running": 64}


def field_rel_l2(a, b):
    """Relative L2 distance of strain fields a, b (loads, 6, n0, n1, n2) on the
    device, off-diagonal tensor components counted twice."""
    import torch
    w = torch.tensor([1.0, 1.0, 1.0, 2.0, 2.0, 2.0], dtype=torch.float64, device=a.device).view(6, 1, 1, 1)
    num = den = 0.0
    for i in range(a.shape[0]):
        num += float(torch.sum(w * (a[i] - b[i]) ** 2))
        den += float(torch.sum(w * b[i] ** 2))
    return (num / den) ** 0.5 if den > 0 else num ** 0.5


def ceff_scaled_diff(c, ref):
    d = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    return float(np.max(np.abs(c - ref) / d))


def kernel_table(prof, nvox, model):
    """Per-category launches, times and (where `model` gives the category's
    algorithmic bytes over the run) achieved GB/s."""
    out = {}
    for c, (n_l, ms, u) in prof.items():
        if n_l == 0:
            continue
        e = {"launches": n_l, "loads": u, "total_ms": round(ms, 3), "avg_ms": round(ms / n_l, 4)}
        if c in model and ms > 0:
            e["alg_bytes"] = round(model[c])
            e["achieved_GBs"] = round(model[c] / (ms * 1e-3) / 1e9, 1)
            e["frac_of_peak"] = round(model[c] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        out[c] = e
    return out


def fp64_models(results, nvox, scheme, order1_index=6):
    """Algorithmic bytes of the FP64 categories over one run of FP64 steps
    (`results`: the per-load result records of every step).  Each step also
    builds the order-1 right-hand side: six displacement transforms of the
    order-0 correctors (x-forward copy 98, x-inverse 3 components 72) and
    the theta transform of g (x-forward 3 components 74, x-inverse accumulate
    144), one FP64 application each."""
    B = BYTES
    xf = xi = 0.0
    apps = 0
    for rs in results:
        xf += 6 * 98.0 + (IDB + 24.0 + F64)
        xi += 6 * (F64 + 24.0) + (F64 + F64 + F64)
        apps += 7
        for l, r in enumerate(rs):
            p_read = B["rhs_P"] if l == order1_index else 0.0
            it = r["iters"]
            if scheme == "cg":
                xf += it * B["cg_xf"] + 2 * (B["ls_xf"] + p_read)
                xi += it * B["cg_xi"] + B["bs_xi"] + B["resid_xi"]
            elif scheme == "cg3":
                xf += B["ls_xf"] + p_read
                xi += B["bs_xi"]
            apps += r["fp64_applications"]
    # two y-passes (forward, inverse) and one z-pass per application
    m = {"ypass_f64": nvox * apps * 2 * B["y64"], "zpass_f64": nvox * apps * B["z64"]}
    if scheme in ("cg", "cg3"):
        m["xfwd_f64"] = nvox * xf
        m["xinv_f64"] = nvox * xi
    if scheme == "cg3":
        its = sum(r["iters"] for rs in results for r in rs)
        starts = sum(1 for rs in results for r in rs if r["iters"] > 0)
        m["xcg3_f64"] = nvox * (its * B["cg3_64"] - starts * B["cg3_64_saving"])
        m["cg3start_f64"] = nvox * starts * B["cg3s_64"]
    return m


def mixed_fp64_models(results, nvox, order1_index=6):
    """Algorithmic bytes of the FP64 sweeps and FP32 projections of the mixed
    runs: per load the first sweep of a solve (x = 0), the later sweeps (with
    the FP32 correction), the order-1 load's reads of its stored right-hand
    side, and the order-1 right-hand-side transforms (see fp64_models)."""
    B = BYTES
    xf = xi = 0.0
    apps = proj = 0
    for rs in results:
        xf += 6 * 98.0 + (IDB + 24.0 + F64)
        xi += 6 * (F64 + 24.0) + (F64 + F64 + F64)
        apps += 7
        for l, r in enumerate(rs):
            sw = r["fp64_applications"]
            later = max(sw - 1, 0)
            xf += B["sweep0_xf"] + later * B["sweep_xf"] + (sw * B["rhs_P"] if l == order1_index else 0.0)
            xi += B["sweep0_xi"] + later * B["sweep_xi"]
            apps += sw
            proj += r["projections"]
    return {"xfwd_f64": nvox * xf, "xinv_f64": nvox * xi, "ypass_f64": nvox * apps * 2 * B["y64"],
            "zpass_f64": nvox * apps * B["z64"], "xfwd_f32": nvox * proj * B["proj_xf"],
            "xinv_f32": nvox * proj * B["proj_xi"]}


def merge_prof(p0, p1):
    return {k: (p0[k][0] + p1[k][0], p0[k][1] + p1[k][1], p0[k][2] + p1[k][2]) for k in p0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--grains", type=int, default=200)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--scheme", default="cg", choices=["cg", "basic"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--inner-tol", type=float, default=1e-3,
                    help="tightest FP32 residual reduction between FP64 reliable updates")
    ap.add_argument("--leg-steps", type=int, default=4, help="timed steps of each comparison leg (at most --steps)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 and FP32-spectrum comparison legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=128)
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (0: the host's cores, at most 16)")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-stream (serving) measurement")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 128^3 random-sphere, FP32-only and fibre measurements")
    ap.add_argument("--no-fibres", action="store_true", help="skip the 512^3 fibre composite")
    ap.add_argument("--fibres-n", type=int, default=512)
    ap.add_argument("--serve-count", type=int, default=512)
    ap.add_argument("--serve-rates", default="40,20", help="request rates (per second) of the serving streams")
    ap.add_argument("--only-serve", action="store_true",
                    help="run the serving measurement alone and print its results (diagnostics, e.g. under a trace)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--no-spectrum16", action="store_true", help="keep the inner solve's spectrum in FP32")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the solver is single-GPU; --gpus {args.gpus} is not supported)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1712_05145_amd import ffth
    from paper_1712_05145_amd import microstructure as M

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    if args.only_serve:
        print(json.dumps({"serving": [serving_run(args.serve_count, float(r), dev)
                                      for r in args.serve_rates.split(",")]}), flush=True)
        return
    t = time.perf_counter()
    phase, lame = M.voronoi_polycrystal(args.n, args.grains, args.seed)
    lam0, mu0 = M.midpoint_reference(lame)
    log(f"microstructure {args.n}^3, {args.grains} grains in {time.perf_counter() - t:.1f}s; C0 = ({lam0:.3f}, {mu0:.3f})")
    nvox = phase.size
    G = default_grad()
    contrast = ffth.ffth_stiffness_contrast(lame=lame)
    h16 = (not args.no_spectrum16 and contrast <= ffth.SPECTRUM16_MAX_CONTRAST
           and nvox >= ffth.SPECTRUM16_MIN_VOXELS)

    def make(precision, order, nloads, scheme=None, spectrum16=None):
        return ffth.Solver(phase, lam0, mu0, lame=lame, nloads=nloads, order=order, scheme=scheme or args.scheme,
                           precision=precision, tol=args.tol, max_iter=50000, inner_tol=args.inner_tol, max_outer=30,
                           check_every=8, autotune=not args.no_autotune,
                           spectrum16=(not args.no_spectrum16) if spectrum16 is None else spectrum16, device=dev)

    # achievable streaming bandwidth on this device (context for the roofline)
    buf_a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    buf_b = torch.empty_like(buf_a)
    buf_b.copy_(buf_a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        buf_b.copy_(buf_a)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * buf_a.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del buf_a, buf_b
    log(f"device copy bandwidth {copy_gbs:.0f} GB/s")

    def step(a, b, e0, e1):
        _, r0 = a.solve_order0(np.eye(6), out=e0)
        _, r1 = b.solve_order1(e0, G, out=e1)
        return r0 + r1

    def run(precision, scheme, spectrum16, warmup, steps, tag):
        """Plans for the step, `warmup` untimed and `steps` timed steps with the
        kernel timing on; returns (times, results, profile, eps0, eps1, tiles)."""
        t = time.perf_counter()
        a = make(precision, 0, 6, scheme, spectrum16)
        b = make(precision, 1, 1, scheme, spectrum16)
        log(f"{tag}: plans (incl. tile autotuning) in {time.perf_counter() - t:.2f}s; tiles {a.tile_variants}, "
            f"loads per launch {a.launch_loads}")
        e0 = a.field(6, 6)
        e1 = b.field(6, 1)
        for w in range(warmup):
            step(a, b, e0, e1)
            log(f"{tag}: warmup {w + 1}/{warmup} done")
        ffth.ffth_profile_enable(a.plan, True)
        ffth.ffth_profile_enable(b.plan, True)
        torch.cuda.synchronize()
        times, results = [], []
        for k in range(steps):
            ts = time.perf_counter()
            results.append(step(a, b, e0, e1))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
            log(f"{tag}: step {k + 1}/{steps}: {times[-1] * 1e3:.1f} ms")
        prof = merge_prof(ffth.ffth_profile_read(a.plan), ffth.ffth_profile_read(b.plan))
        bad = [r for rs in results for r in rs if r["status"] != 0]
        if bad:
            raise SystemExit(f"{tag}: solve failed: {bad[0]}")
        tiles = a.tile_variants + a.launch_loads   # 8 tile variants, loads per launch FP32 / FP64
        # order-1 right-hand side alone (displacements of the six correctors,
        # pointwise terms, theta), outside the timed steps
        torch.cuda.synchronize()
        tr = time.perf_counter()
        b.order1_rhs(e0, G.reshape(18))
        torch.cuda.synchronize()
        rhs_ms = (time.perf_counter() - tr) * 1e3
        a.close()
        b.close()
        return times, results, prof, e0, e1, tiles, rhs_ms

    times, results, prof, eps0, eps1, tiles, rhs_ms = run("mixed", args.scheme, None, args.warmup, args.steps, "mixed")
    elapsed = sum(times)
    inner = sum(r["iters"] for rs in results for r in rs)
    fp64_apps = sum(r["fp64_applications"] for rs in results for r in rs)
    proj = sum(r["projections"] for rs in results for r in rs)
    value = nvox * (inner + proj + fp64_apps) / elapsed
    ms_step = elapsed / args.steps * 1e3
    ceff = np.array([r["mean_stress"] for r in results[-1][:6]]).T

    # roofline of the dominant kernel.  Units = loads a category's launches
    # really processed: a launch still carries loads that converged since the
    # last read-back (their blocks exit at once), so the inner-loop kernels
    # take their counts from the solver's own iteration counts instead.
    starts = prof["cg3start_f32"][2]
    real_units = {"xcg3_f32": inner, "ypass_f32": 2 * (inner + proj), "zpass_f32": inner + proj}
    prof = {k: (v[0], v[1], real_units.get(k, v[2])) for k, v in prof.items()}
    ab = alg_bytes_per_voxel(h16)

    def alg_bytes(c, u):
        if c == "ypass_f32":
            return nvox * (inner * (ab["yf"] + ab["yi"]) + proj * 96.0)
        if c == "zpass_f32":
            return nvox * (inner * ab["z"] + proj * 48.0)
        if c == "xcg3_f32":
            return nvox * (inner * ab["xcg3"] - XCG3_START_SAVING * starts)
        return nvox * ab["start"] * u

    cat = max(ALG_CATEGORIES, key=lambda c: prof[c][1])
    launches, tot_ms, units = prof[cat]
    bytes_total = alg_bytes(cat, units)
    achieved = bytes_total / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    model = {c: alg_bytes(c, prof[c][2]) for c in ALG_CATEGORIES}
    model.update(mixed_fp64_models(results, nvox))
    kernels = kernel_table(prof, nvox, model)
    for c in ALG_CATEGORIES:
        if c in kernels and prof[c][2]:
            kernels[c]["alg_bytes_per_voxel_per_load"] = round(model[c] / (nvox * prof[c][2]), 2)
    # the committed counters were taken with the binary16 forward spectrum:
    # HBM bytes per algorithmic byte there, times this run's algorithmic
    # bytes per launch
    t_ratio = measured_traffic(cat) if h16 else None
    upl = units / max(launches, 1)
    roofline = {"bound": "hbm", "kernel": cat, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if t_ratio is None else round(t_ratio * bytes_total / max(launches, 1)),
                "traffic_ratio": t_ratio, "alg_bytes_per_launch": round(bytes_total / max(launches, 1)),
                "alg_bytes_per_voxel_per_load": round(bytes_total / (nvox * max(units, 1)), 2),
                "units_per_launch": round(upl, 3),
                "avg_launch_ms": round(tot_ms / max(launches, 1), 4),
                "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}

    # one FP32 inner iteration of one load over its four passes (fused CG pass,
    # forward y, z with the Green operator, inverse y): algorithmic bytes per
    # voxel and the per-load times of the same timed steps
    it_ms = {c: prof[c][1] / max(prof[c][2], 1) for c in ("xcg3_f32", "ypass_f32", "zpass_f32")}
    it_ms_total = it_ms["xcg3_f32"] + 2 * it_ms["ypass_f32"] + it_ms["zpass_f32"]
    it_bpv = ab["xcg3"] + ab["yf"] + ab["yi"] + ab["z"]
    inner_iteration = {"alg_bytes_per_voxel": it_bpv, "ms_per_load": round(it_ms_total, 4),
                       "achieved_GBs": round(it_bpv * nvox / (it_ms_total * 1e-3) / 1e9, 1) if it_ms_total > 0 else None,
                       "frac_of_peak": round(it_bpv * nvox / (it_ms_total * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                       if it_ms_total > 0 else None}

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "voxel-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16-spectrum/f32+f64" if h16 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"voronoi{args.n}-order0x6+order1", "grid": [args.n] * 3, "grains": args.grains,
                   "seed": args.seed, "scheme": args.scheme, "precision": "mixed", "tol": args.tol,
                   "loads_order0": 6, "loads_order1": 1, "parallelism": "single-gpu",
                   "inner_spectrum": "binary16 forward, FP32 after the Green operator" if h16 else "FP32",
                   "stiffness_contrast": round(contrast, 2)},
        "voxel_iters": {"fp32_inner": int(inner * nvox / args.steps), "fp32_projection": int(proj * nvox / args.steps),
                        "fp64": int(fp64_apps * nvox / args.steps)},
        "iters_per_step": {"fp32_inner": inner // args.steps, "fp32_projections": proj // args.steps,
                           "fp64_applications": fp64_apps // args.steps},
        "latency_ms": {"p50": round(float(np.percentile(times, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(times, 99)) * 1e3, 2), "over": "timed steps"},
        "order1_rhs_ms": round(rhs_ms, 2),
        "roofline": roofline,
        "inner_iteration": inner_iteration,
        "kernels": kernels,
        "tile_variants": dict(zip(["xfwd_f32", "xfwd_f64", "ypass_f32", "ypass_f64", "zpass_f32", "zpass_f64",
                                   "xinv_f32", "xinv_f64", "loads_per_launch_f32", "loads_per_launch_f64"],
                                  tiles)),
    }
    torch.cuda.empty_cache()

    lw, ls = min(args.warmup, 1), max(1, min(args.steps, args.leg_steps))

    def compare(tag, precision, scheme, spectrum16, models=None):
        tl, rl, pl, e0, e1, tl_tiles, rhs = run(precision, scheme, spectrum16, lw, ls, tag)
        ms = sum(tl) / len(tl) * 1e3
        c = np.array([r["mean_stress"] for r in rl[-1][:6]]).T
        m1 = np.array(rl[-1][6]["mean_stress"])
        m1_ref = np.array(results[-1][6]["mean_stress"])
        apps = sum(r["fp64_applications"] + r["projections"] + (r["iters"] if precision != "fp64" else 0)
                   for r in rl[-1])
        out = {"ms_per_step": round(ms, 2), "steps": ls, "warmup": lw,
               "iters_per_step": sum(r["iters"] for r in rl[-1]),
               "fp64_applications_per_step": sum(r["fp64_applications"] for r in rl[-1]),
               "voxel_iters_per_s": round(nvox * apps / (ms * 1e-3), 1),
               "speedup_mixed_vs_this": round(ms / ms_step, 3),
               "ceff_max_scaled_diff_vs_mixed": ceff_scaled_diff(ceff, c),
               "order0_field_rel_l2_vs_mixed": field_rel_l2(eps0, e0),
               "order1_field_rel_l2_vs_mixed": field_rel_l2(eps1, e1),
               "order1_mean_stress_max_diff_vs_mixed": float(np.abs(m1 - m1_ref).max() / np.abs(m1_ref).max()),
               "residuals": [r["residual"] for r in rl[-1]], "tiles": tl_tiles, "order1_rhs_ms": round(rhs, 2)}
        if models is not None:
            out["kernels"] = kernel_table(pl, nvox, models(rl))
        log(f"{tag}: {ms:.1f} ms per step ({ms / ms_step:.2f}x the mixed step), "
            f"order-1 field vs mixed {out['order1_field_rel_l2_vs_mixed']:.2e}")
        del e0, e1
        torch.cuda.empty_cache()
        return out

    if not args.no_fp64:
        if h16:
            line["fp32_spectrum_path"] = compare(
                "fp32-spectrum", "mixed", args.scheme, False,
                lambda rl: dict(mixed_fp64_models(rl, nvox)))
        line["fp64_path"] = compare("fp64-cg", "fp64", "cg", False, lambda rl: fp64_models(rl, nvox, "cg"))
        line["fp64_three_term_path"] = compare("fp64-cg3", "fp64", "cg3", False,
                                               lambda rl: fp64_models(rl, nvox, "cg3"))
        line["bicgstab_fp64_path"] = compare("fp64-bicgstab", "fp64", "bicgstab", False)
        line["speedups"] = {
            "mixed_vs_fp64_two_term_cg": line["fp64_path"]["speedup_mixed_vs_this"],
            "mixed_vs_fp64_three_term_cg": line["fp64_three_term_path"]["speedup_mixed_vs_this"],
            "mixed_vs_fp64_bicgstab": line["bicgstab_fp64_path"]["speedup_mixed_vs_this"],
            "note": "the three-term FP64 CG runs the same fused passes as the mixed path's inner solve, "
                    "so mixed_vs_fp64_three_term_cg is the precision-only speedup"}
        if h16:
            line["speedups"]["binary16_spectrum_vs_fp32_spectrum"] = line["fp32_spectrum_path"]["speedup_mixed_vs_this"]
    if not args.no_configs:
        line["fp32_only"] = fp32_only_run(dev, phase, lame, lam0, mu0, eps0, ceff)
    del eps0, eps1
    torch.cuda.empty_cache()
    if not args.no_configs:
        line["spheres128"] = spheres128_run(dev)
        if not args.no_fibres:
            line["fibres512"] = fibres_run(dev, args.fibres_n)
    if not args.no_serve:
        line["serving"] = [serving_run(args.serve_count, float(r), dev) for r in args.serve_rates.split(",")]
    if not args.no_cpu:
        apps_fp64 = line.get("fp64_path", {}).get("fp64_applications_per_step")
        workers = args.cpu_workers or max(1, min(16, len(os.sched_getaffinity(0))))
        line["cpu_baseline"] = cpu_baseline(args.cpu_n, args.grains, args.seed, apps_fp64, args.n, workers)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
