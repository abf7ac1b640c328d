"""Serving driver over the libffth request server (ffth_server_* in
include/ffth.h): a caller-owned HBM arena, admission by memory (least work
first, with a bound on how often a request may be passed over), continuous
batching of running solves on per-grid streams, and a wall-clock replay of a
Poisson request stream reporting p50/p99 latency beside throughput.

All solving happens in libffth; this module allocates the arena and the
per-request phase arrays with torch and keeps them alive while requests run.
"""
import ctypes
import time

import numpy as np

from . import ffth


class Server:
    def __init__(self, budget_bytes, max_running=32, tol=1e-8, inner_tol=1e-3, check_every=8, max_iter=20000,
                 device="cuda:0", stream=None, spectrum16=True):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.opts = ffth.make_opts("cg", "mixed", tol=tol, max_iter=max_iter, inner_tol=inner_tol,
                                   check_every=check_every, spectrum16=spectrum16)
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.srv = ffth.ffth_server_create(ffth._dptr(self.arena), int(budget_bytes), self.opts, max_running,
                                           ctypes.c_void_p(self.stream.cuda_stream))
        self.live = {}

    def request_bytes(self, n, nphases, nloads=6):
        return ffth.ffth_request_bytes(n, nphases, nloads, self.opts)

    def submit(self, phase, lame, lam0, mu0, E, voigt21=None):
        """One request: phase ids on the grid, the phases' (lambda, mu) pairs
        (lame) or, with lame None, their 21 Voigt coefficients (voigt21)."""
        torch = self.torch
        ph = phase if not isinstance(phase, np.ndarray) else torch.from_numpy(
            np.ascontiguousarray(phase.astype(np.uint16)).view(np.int16))
        ph = ph.to(self.device).contiguous()
        pr = ffth.ffth_problem()
        pr.n = (ctypes.c_int32 * 3)(*ph.shape)
        if lame is not None:
            lame_a, lame_p = ffth._darr(lame)
            pr.nphases = lame_a.reshape(-1, 2).shape[0]
            pr.lame, pr.stiffness = lame_p, None
        else:
            lame_a, v_p = ffth._darr(np.asarray(voigt21, np.float64).reshape(-1, 21))
            pr.nphases = lame_a.shape[0]
            pr.lame, pr.stiffness = None, v_p
        pr.phase = ph.data_ptr()
        pr.lambda0, pr.mu0 = lam0, mu0
        E = np.asarray(E, np.float64).reshape(-1, 6)
        rid = ffth.ffth_submit(self.srv, pr, E)
        self.live[rid] = (ph, lame_a, E.shape[0], int(np.prod(ph.shape)))
        return rid

    def step(self):
        return ffth.ffth_server_step(self.srv)

    def poll(self, rid):
        nl = self.live[rid][2]
        st, res = ffth.ffth_poll(self.srv, rid, nl)
        if st != ffth.FFTH_ERR_BUSY:
            self.live.pop(rid, None)
        return st, res

    def stats(self):
        """Inner iterations run as multi-size launches and the most distinct
        grids one such launch carried."""
        return ffth.ffth_server_stats(self.srv)

    def cancel(self, rid):
        ffth.ffth_cancel(self.srv, rid)

    def close(self):
        if getattr(self, "srv", None) is not None:
            ffth.ffth_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server, stream, inputs, loads=None, time_scale=1.0, on_done=None):
    """Replay `stream` (dicts with 'id', 'arrival' seconds) in wall-clock time.

    inputs[i] = (phase, lame, lam0, mu0) for request i.  Each request solves the
    six unit loads unless `loads` is given.  Returns per-request records and
    aggregate statistics (latency = completion - arrival)."""
    E = np.eye(6) if loads is None else np.asarray(loads, np.float64)
    order = sorted(stream, key=lambda r: r["arrival"])
    pending = list(order)
    inflight = {}
    records = []
    t0 = time.perf_counter()
    while pending or inflight:
        now = time.perf_counter() - t0
        while pending and pending[0]["arrival"] * time_scale <= now:
            req = pending.pop(0)
            ph, lame, lam0, mu0 = inputs[req["id"]]
            rid = server.submit(ph, lame, lam0, mu0, E)
            inflight[rid] = (req, req["arrival"] * time_scale, int(np.prod(np.shape(ph))))
        if not inflight:
            time.sleep(max(0.0, pending[0]["arrival"] * time_scale - (time.perf_counter() - t0)))
            continue
        server.step()
        tnow = time.perf_counter() - t0
        for rid in list(inflight):
            st, res = server.poll(rid)
            if st == ffth.FFTH_ERR_BUSY:
                continue
            req, arr, nvox = inflight.pop(rid)
            rec = {"id": req["id"], "n": req.get("n"), "status": st, "arrival": arr, "done": tnow,
                   "latency": tnow - arr, "results": res,
                   "voxel_iters": nvox * sum(r["iters"] + r["projections"] + r["fp64_applications"] for r in res)
                   if res else 0}
            records.append(rec)
            if on_done:
                on_done(rec)
    makespan = time.perf_counter() - t0
    lat = np.array([r["latency"] for r in records])
    vi = sum(r["voxel_iters"] for r in records)
    stats = {"requests": len(records), "makespan_s": makespan,
             "latency_p50_ms": float(np.percentile(lat, 50) * 1e3), "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
             "voxel_iters_per_s": vi / makespan, "failed": sum(1 for r in records if r["status"] != 0)}
    return records, stats
