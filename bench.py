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
#   fused three-term CG    spectrum, r_k, x_k, r_k-1, x_k-1, phase read;
#   x-pass                 r_k+1, x_k+1, spectrum written            24*5+2+24*3
#   start pass of a solve  r_0, phase read; spectrum written          24+2+24
# With the binary16 forward spectrum of the inner solve, every write of the
# spectrum before the spectral operator and every read of it up to there is
# 12 B: forward y-pass 12+12, z-pass 12+24, fused pass 24*5+2+24*2+12, start
# pass 24+2+12; the inverse y-pass (24+24) and the projection passes stay FP32.
# The first iteration of each inner solve reads neither x_k nor r_k-1, x_k-1
# (x_0 = 0, omega = 1) and the second does not read x_k-1: per started solve
# the fused kernel moves 72 + 24 B/voxel less than a full iteration.  The
# model subtracts both for every start (a lower bound on the bytes moved when
# a solve stops after one iteration).  The FP32 x-forward / x-inverse
# categories hold the projection passes only and are reported without a model.
ALG_CATEGORIES = ("ypass_f32", "zpass_f32", "xcg3_f32", "cg3start_f32")
XCG3_START_SAVING = 96.0


def alg_bytes_per_voxel(h16):
    """Bytes per voxel of (forward y, inverse y, z, fused CG pass, start pass)
    in the inner solve; projection passes move 48 B in each y- and z-pass."""
    if h16:
        return {"yf": 24.0, "yi": 48.0, "z": 36.0, "xcg3": 182.0, "start": 38.0}
    return {"yf": 48.0, "yi": 48.0, "z": 48.0, "xcg3": 194.0, "start": 50.0}


def measured_traffic(cat):
    """HBM bytes per load-launch of kernel category `cat` from the committed
    counter summary, or None when the kernel sources changed since it was taken."""
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
        if line.startswith(f"traffic-bytes-per-load-launch {cat}:"):
            return float(line.split(":")[1])
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def default_grad():
    g = np.zeros((6, 3))
    g[0, 0] = 1.0      # dE_11/dY_1
    g[1, 1] = 1.0      # dE_22/dY_2
    return g.reshape(1, 18)


def cpu_baseline(n_sample, grains, seed):
    """The FP64 oracle, one operator application on the same generator at n_sample^3."""
    from threadpoolctl import threadpool_limits

    from oracle import homogenization as H
    from paper_1712_05145_amd import microstructure as M
    phase, lame = M.voronoi_polycrystal(n_sample, grains, seed)
    lam0, mu0 = M.midpoint_reference(lame)
    prob = H.make_problem(phase, lam0, mu0, lame=lame)
    x = np.random.default_rng(0).standard_normal((3, 3) + phase.shape)
    x = 0.5 * (x + np.swapaxes(x, 0, 1))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        prob.apply_A(x)
        dt = time.perf_counter() - t0
    return {"value": phase.size / dt, "unit": "voxel-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 operator application (FFT, Green operator, inverse FFT) of the oracle on the "
                      f"{n_sample}^3 Voronoi polycrystal of the same generator, single thread, {dt:.1f} s"}


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
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=128)
    ap.add_argument("--no-serve", action="store_true", help="skip the request-stream (serving) measurement")
    ap.add_argument("--no-configs", action="store_true", help="skip the 128^3 random-sphere measurement")
    ap.add_argument("--serve-count", type=int, default=512)
    ap.add_argument("--serve-rate", type=float, default=40.0)
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
    t = time.perf_counter()
    phase, lame = M.voronoi_polycrystal(args.n, args.grains, args.seed)
    lam0, mu0 = M.midpoint_reference(lame)
    log(f"microstructure {args.n}^3, {args.grains} grains in {time.perf_counter() - t:.1f}s; C0 = ({lam0:.3f}, {mu0:.3f})")
    nvox = phase.size
    G = default_grad()

    def make(precision, order, nloads, scheme=None):
        return ffth.Solver(phase, lam0, mu0, lame=lame, nloads=nloads, order=order, scheme=scheme or args.scheme,
                           precision=precision, tol=args.tol, max_iter=50000, inner_tol=args.inner_tol, max_outer=30,
                           check_every=8, autotune=not args.no_autotune, spectrum16=not args.no_spectrum16,
                           device=dev)

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

    t = time.perf_counter()
    s0 = make("mixed", 0, 6)
    s1 = make("mixed", 1, 1)
    log(f"plans (incl. tile autotuning) in {time.perf_counter() - t:.2f}s; tiles {s0.tile_variants}")
    eps0 = s0.field(6, 6)
    eps1 = s1.field(6, 1)

    def step(a, b, e0, e1):
        _, r0 = a.solve_order0(np.eye(6), out=e0)
        _, r1 = b.solve_order1(e0, G, out=e1)
        return r0 + r1

    for w in range(args.warmup):
        step(s0, s1, eps0, eps1)
        log(f"warmup {w + 1}/{args.warmup} done")
    ffth.ffth_profile_enable(s0.plan, True)
    ffth.ffth_profile_enable(s1.plan, True)
    torch.cuda.synchronize()
    times, results = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        results.append(step(s0, s1, eps0, eps1))
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        log(f"step {k + 1}/{args.steps}: {times[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof0 = ffth.ffth_profile_read(s0.plan)
    prof1 = ffth.ffth_profile_read(s1.plan)
    ffth.ffth_profile_enable(s0.plan, False)
    ffth.ffth_profile_enable(s1.plan, False)

    inner = sum(r["iters"] for rs in results for r in rs)
    fp64_apps = sum(r["fp64_applications"] for rs in results for r in rs)
    proj = sum(r["projections"] for rs in results for r in rs)
    bad = [r for rs in results for r in rs if r["status"] != 0]
    if bad:
        raise SystemExit(f"solve failed: {bad[0]}")
    value = nvox * (inner + proj + fp64_apps) / elapsed
    ms_step = elapsed / args.steps * 1e3
    ceff = np.array([r["mean_stress"] for r in results[-1][:6]]).T

    # roofline of the dominant kernel.  Units = loads a category's launches
    # really processed: a launch still carries loads that converged since the
    # last read-back (their blocks exit at once), so the inner-loop kernels
    # take their counts from the solver's own iteration counts instead.
    prof = {k: (prof0[k][0] + prof1[k][0], prof0[k][1] + prof1[k][1], prof0[k][2] + prof1[k][2]) for k in prof0}
    starts = prof["cg3start_f32"][2]
    real_units = {"xcg3_f32": inner, "ypass_f32": 2 * (inner + proj), "zpass_f32": inner + proj}
    prof = {k: (v[0], v[1], real_units.get(k, v[2])) for k, v in prof.items()}

    ab = alg_bytes_per_voxel(not args.no_spectrum16)

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
    kernels = {}
    for c in prof:
        n_l, ms, u = prof[c]
        entry = {"launches": n_l, "loads": u, "total_ms": round(ms, 3),
                 "avg_ms": round(ms / n_l, 4) if n_l else None,
                 "ms_per_load": round(ms / u, 4) if u else None}
        if c in ALG_CATEGORIES and ms > 0:
            entry["alg_bytes_per_voxel_per_load"] = round(alg_bytes(c, u) / (nvox * u), 2)
            entry["achieved_GBs"] = round(alg_bytes(c, u) / (ms * 1e-3) / 1e9, 1)
        kernels[c] = entry
    # the committed counters were taken with the binary16 forward spectrum
    t_unit = None if args.no_spectrum16 else measured_traffic(cat)
    upl = units / max(launches, 1)
    roofline = {"bound": "hbm", "kernel": cat, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if t_unit is None else round(t_unit * upl),
                "traffic_per_load_launch": t_unit, "alg_bytes_per_launch": round(bytes_total / max(launches, 1)),
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
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"voronoi{args.n}-order0x6+order1", "grid": [args.n] * 3, "grains": args.grains,
                   "seed": args.seed, "scheme": args.scheme, "precision": "mixed", "tol": args.tol,
                   "loads_order0": 6, "loads_order1": 1, "parallelism": "single-gpu"},
        "voxel_iters": {"fp32_inner": int(inner * nvox / args.steps), "fp32_projection": int(proj * nvox / args.steps),
                        "fp64": int(fp64_apps * nvox / args.steps)},
        "iters_per_step": {"fp32_inner": inner // args.steps, "fp32_projections": proj // args.steps,
                           "fp64_applications": fp64_apps // args.steps},
        "latency_ms": {"p50": round(float(np.percentile(times, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(times, 99)) * 1e3, 2), "over": "timed steps"},
        "roofline": roofline,
        "inner_iteration": inner_iteration,
        "kernels": kernels,
        "tile_variants": dict(zip(["xfwd_f32", "xfwd_f64", "ypass_f32", "ypass_f64", "zpass_f32", "zpass_f64",
                                   "xinv_f32", "xinv_f64"], s0.tile_variants)),
    }
    del s0, s1
    torch.cuda.empty_cache()

    if not args.no_fp64:
        f0 = make("fp64", 0, 6)
        f1 = make("fp64", 1, 1)
        e0 = f0.field(6, 6)
        e1 = f1.field(6, 1)
        torch.cuda.synchronize()
        tf = time.perf_counter()
        rf = step(f0, f1, e0, e1)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - tf
        it64 = sum(r["iters"] for r in rf)
        c64 = np.array([r["mean_stress"] for r in rf[:6]]).T
        diff = np.abs(ceff - c64) / np.sqrt(np.outer(np.diag(c64), np.diag(c64)))
        apps64 = sum(r["fp64_applications"] for r in rf)
        line["fp64_path"] = {"ms_per_step": round(t64 * 1e3, 2), "iters_per_step": it64,
                             "voxel_iters_per_s": round(nvox * apps64 / t64, 1),
                             "speedup_mixed_vs_fp64": round(t64 * 1e3 / ms_step, 3),
                             "ceff_max_scaled_diff": float(diff.max()),
                             "residuals": [r["residual"] for r in rf]}
        log(f"fp64 step {t64 * 1e3:.1f} ms, C_eff diff {diff.max():.2e}")
        del f0, f1, e0, e1
        torch.cuda.empty_cache()
        # the paper's Krylov method (BiCGSTAB) in FP64 on the same step
        b0 = make("fp64", 0, 6, "bicgstab")
        b1 = make("fp64", 1, 1, "bicgstab")
        e0 = b0.field(6, 6)
        e1 = b1.field(6, 1)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        rb = step(b0, b1, e0, e1)
        torch.cuda.synchronize()
        tbi = time.perf_counter() - tb
        cb = np.array([r["mean_stress"] for r in rb[:6]]).T
        diffb = np.abs(ceff - cb) / np.sqrt(np.outer(np.diag(cb), np.diag(cb)))
        appsb = sum(r["fp64_applications"] for r in rb)
        line["bicgstab_fp64_path"] = {"ms_per_step": round(tbi * 1e3, 2),
                                      "iters_per_step": sum(r["iters"] for r in rb),
                                      "fp64_applications_per_step": appsb,
                                      "voxel_iters_per_s": round(nvox * appsb / tbi, 1),
                                      "speedup_mixed_cg_vs_bicgstab_fp64": round(tbi * 1e3 / ms_step, 3),
                                      "ceff_max_scaled_diff": float(diffb.max()),
                                      "residuals": [r["residual"] for r in rb]}
        log(f"bicgstab fp64 step {tbi * 1e3:.1f} ms, C_eff diff {diffb.max():.2e}")
        del b0, b1, e0, e1
        torch.cuda.empty_cache()
    if not args.no_configs:
        line["spheres128"] = spheres128_run(dev)
    if not args.no_serve:
        line["serving"] = serving_run(args.serve_count, args.serve_rate, dev)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_n, args.grains, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
