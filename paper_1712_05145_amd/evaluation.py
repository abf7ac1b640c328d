"""The paper's evaluation (Sec. 4) on the GPU path: Hashin's coated circular
inclusion (core radius 0.25, coating radius 0.4, E = 100 / 1000 / 453.685,
nu = 0.3, plane stress) on (1, n, n) grids, tolerance 1e-6, FP64.

  grid sweep (Sec. 4, iterations and time against n):  n = 8 ... 1024
  contrast sweep (iterations and time against the contrast of core and
      coating, 64 x 64): coating modulus varied, core fixed, matrix modulus
      kept neutral for each pair
  time ratios (Sec. 4, Table 1): second-order over first-order time

First-order problem: the order-0 solve for the macroscopic strain E = Id of
the plane (E22 = E33 = 1).  Second-order problem: the three in-plane order-0
correctors (unit loads E22, E33, 2 E23) solved one after another, then the
order-1 right-hand side and solve for the paper's gradient load, which in the
(x2, x3) plane reads (grad E)_222 = (grad E)_333 = 1.  Schemes: the Basic
Scheme, conjugate gradients on eq. (6), and BiCGSTAB on eq. (6) (the routine
the paper's "CG-version" ran; one BiCGSTAB iteration is two operator
applications).

Run:  python -m paper_1712_05145_amd.evaluation [--out FILE] [--sizes ...]
"""
import argparse
import json
import os
import time

import numpy as np

from . import ffth
from . import microstructure as M

IN_PLANE = np.array([[0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0], [0, 0, 0, 1, 0, 0]], dtype=float)
IDENTITY = np.array([0, 1, 1, 0, 0, 0], dtype=float)


def paper_gradient():
    g = np.zeros((6, 3))
    g[1, 1] = g[2, 2] = 1.0          # d E22 / d Y2 = d E33 / d Y3 = 1
    return g.reshape(1, 18)


def run_case(phase, lame, scheme, tol=1e-6, precision="fp64", max_iter=400000):
    """Times and iteration counts of the first- and second-order problems."""
    import torch
    lam0, mu0 = M.midpoint_reference(lame)
    kw = dict(lame=lame, scheme=scheme, precision=precision, tol=tol, max_iter=max_iter,
              check_every=64 if scheme == "basic" else 8)
    s0 = ffth.Solver(phase, lam0, mu0, nloads=1, **kw)
    s1 = ffth.Solver(phase, lam0, mu0, nloads=1, order=1, **kw)
    e_first = s0.field(6, 1)
    corr = torch.zeros((6, 6) + tuple(phase.shape), dtype=torch.float64, device=e_first.device)
    e_second = s1.field(6, 1)
    # warm-up (tile tuning, first launches)
    s0.solve_order0(IDENTITY, out=e_first)
    torch.cuda.synchronize()

    t = time.perf_counter()
    _, r_first = s0.solve_order0(IDENTITY, out=e_first)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t

    t = time.perf_counter()
    it_corr = 0
    for j, e in enumerate(IN_PLANE):              # one first-order problem after another
        _, r = s0.solve_order0(e, out=corr[j + 1:j + 2])
        it_corr += r[0]["iters"]
    _, r_second = s1.solve_order1(corr, paper_gradient(), out=e_second)
    torch.cuda.synchronize()
    t_second = time.perf_counter() - t
    s0.close()
    s1.close()
    return {"first": {"iters": r_first[0]["iters"], "seconds": t_first, "status": r_first[0]["status"]},
            "second": {"iters": r_second[0]["iters"], "corrector_iters": it_corr, "seconds": t_second,
                       "status": r_second[0]["status"]},
            "ratio": t_second / t_first if t_first > 0 else None}


def grid_sweep(sizes, schemes=("basic", "cg", "bicgstab")):
    rows = []
    for n in sizes:
        phase, lame = M.hashin_2d(n)
        for scheme in schemes:
            r = run_case(phase, lame, scheme)
            r.update(n=n, scheme=scheme)
            rows.append(r)
            print(json.dumps(r), flush=True)
    return rows


def contrast_sweep(contrasts, n=64, schemes=("basic", "cg", "bicgstab")):
    rows = []
    for c in contrasts:
        phase, lame = M.hashin_2d_contrast(n, c)
        for scheme in schemes:
            r = run_case(phase, lame, scheme)
            r.update(contrast=c, scheme=scheme, n=n)
            rows.append(r)
            print(json.dumps(r), flush=True)
    return rows


TABLE1_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                           "table1_time_ratios.json")


def paper_table1(path=TABLE1_PATH):
    """{(n, scheme): ratio} of the paper's Table 1 (Sec. 4: second- over
    first-order time); the paper's CG version ran a BiCGSTAB routine, so its
    column stands beside both Krylov rows here.  Empty if the file is absent."""
    if not os.path.exists(path):
        return {}
    t = json.load(open(path))
    out = {}
    for n, bs, cg in zip(t["n"], t["basic_scheme"], t["cg_version"]):
        out[(n, "basic")] = bs
        out[(n, "cg")] = cg
        out[(n, "bicgstab")] = cg
    return out


def write_markdown(path, grid, contrast, cmd):
    name = {"basic": "Basic Scheme", "cg": "CG", "bicgstab": "BiCGSTAB"}
    paper = paper_table1()
    with open(path, "w") as f:
        f.write("# Sec. 4 evaluation on the GPU path: Hashin's coated inclusion, plane stress, (1, n, n) grids\n\n")
        f.write("Command (from the repository root on one MI355X):\n\n```\n" + cmd + "\n```\n\n")
        f.write("FP64, tolerance 1e-6, reference medium at the midpoint of the phase moduli.  First order: "
                "E = Id of the plane.  Second order: three in-plane correctors one after another, then the "
                "order-1 right-hand side and solve for (grad E)_222 = (grad E)_333 = 1.  Times are wall "
                "clock around each problem (device synchronised), after one warm-up solve; small grids are "
                "bound by launch latency, not by the device.\n\n")
        f.write("## Iterations and time against n\n\n")
        f.write("The last column is the paper's Table 1 ratio for the same n (MATLAB on unstated hardware; "
                "its CG version is a BiCGSTAB routine): context, not a target.\n\n")
        f.write("| n | scheme | order-0 iters | order-0 ms | order-1 iters | order-1 ms (incl. 3 correctors) "
                "| ratio | Table 1 |\n|---|---|---|---|---|---|---|---|\n")
        for r in grid:
            pv = paper.get((r["n"], r["scheme"]))
            f.write(f"| {r['n']} | {name[r['scheme']]} | {r['first']['iters']} | {r['first']['seconds'] * 1e3:.2f} "
                    f"| {r['second']['iters']} | {r['second']['seconds'] * 1e3:.2f} | {r['ratio']:.3f} "
                    f"| {'-' if pv is None else f'{pv:.4f}'} |\n")
        f.write("\n## Iterations and time against the contrast (64 x 64)\n\n")
        f.write("Core modulus fixed, coating modulus = contrast x core, matrix modulus neutral for the pair.\n\n")
        f.write("| contrast | scheme | order-0 iters | order-0 ms | order-1 iters | order-1 ms | ratio |\n"
                "|---|---|---|---|---|---|---|\n")
        for r in contrast:
            f.write(f"| {r['contrast']:g} | {name[r['scheme']]} | {r['first']['iters']} "
                    f"| {r['first']['seconds'] * 1e3:.2f} | {r['second']['iters']} "
                    f"| {r['second']['seconds'] * 1e3:.2f} | {r['ratio']:.3f} |\n")
        f.write("\nMachine-readable rows:\n\n```\n")
        for r in grid + contrast:
            f.write(json.dumps(r) + "\n")
        f.write("```\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", type=int, nargs="*", default=[8, 16, 32, 64, 128, 256, 512, 1024])
    ap.add_argument("--contrasts", type=float, nargs="*",
                    default=[1e-4, 1e-3, 1e-2, 1e-1, 1e1, 1e2, 1e3, 1e4])
    ap.add_argument("--out", default=None, help="markdown summary to write")
    args = ap.parse_args()
    grid = grid_sweep(args.sizes)
    contrast = contrast_sweep(args.contrasts)
    if args.out:
        cmd = "python -m paper_1712_05145_amd.evaluation --out " + args.out
        write_markdown(args.out, grid, contrast, cmd)


if __name__ == "__main__":
    main()
