"""Serving (continuous batching under an HBM budget): results are identical
alone and in a mix, admission respects the budget, cancellation and
oversize requests are handled."""
import numpy as np
import pytest

from paper_1712_05145_amd import ffth
from paper_1712_05145_amd import microstructure as M
from tests._gpu import require_gpu

pytestmark = pytest.mark.gpu


def _req(n, frac, contrast, seed):
    phase, lame = M.overlapping_spheres(n, frac, contrast, seed)
    lam0, mu0 = M.midpoint_reference(lame)
    return phase, lame, lam0, mu0


def _drain(srv, ids):
    out = {}
    for _ in range(100000):
        srv.step()
        for rid in list(ids):
            st, res = srv.poll(rid)
            if st != ffth.FFTH_ERR_BUSY:
                out[rid] = (st, res)
                ids.remove(rid)
        if not ids:
            return out
    raise AssertionError("server did not drain")


def _alone(req):
    from paper_1712_05145_amd.serving import Server
    srv = Server(16 << 30, max_running=8)
    rid = srv.submit(*req, np.eye(6))
    out = _drain(srv, [rid])[rid]
    srv.close()
    return out


def test_alone_equals_mix_and_plan_path():
    """Requests that share launches give bit-identical results alone and in
    the mix: a and b (128^3, stiffness contrast within the binary16 limit)
    share every binary16 launch; c and e (64^3, FP32 spectrum) share every
    launch of their group; d (128^3, above the contrast limit, so FP32
    spectrum), f (48^3), g (32^3) and h (16^3) have groups of their own.  The
    five grids take the server's four streams in order of admission, so h
    shares the stream of c and e, and their inner iterations run as one
    launch per pass across the two grid sizes.  a and c are also identical
    through the plan path with autotuning off (the server keeps the default
    tiles on grids of its multi-size launches)."""
    torch = require_gpu()
    from paper_1712_05145_amd.serving import Server
    a = _req(128, 0.25, 20.0, 1)
    b = _req(128, 0.3, 12.0, 6)
    c = _req(64, 0.3, 200.0, 2)
    d = _req(128, 0.35, 400.0, 4)
    e = _req(64, 0.1, 5.0, 5)
    f = _req(48, 0.2, 10.0, 3)
    g = _req(32, 0.25, 30.0, 7)
    h = _req(16, 0.3, 15.0, 8)
    lim = ffth.SPECTRUM16_MAX_CONTRAST
    assert ffth.ffth_stiffness_contrast(lame=a[1]) <= lim and ffth.ffth_stiffness_contrast(lame=b[1]) <= lim
    assert ffth.ffth_stiffness_contrast(lame=d[1]) > lim
    shared = {"a": a, "b": b, "c": c, "d": d, "e": e, "f": f, "g": g, "h": h}
    alone = {k: _alone(r) for k, r in shared.items()}
    s2 = Server(16 << 30, max_running=8)
    order = [("c", c), ("f", f), ("a", a), ("d", d), ("g", g), ("h", h), ("e", e), ("b", b)]
    ids = {k: s2.submit(*r, np.eye(6)) for k, r in order}
    mixed = _drain(s2, list(ids.values()))
    stats = s2.stats()
    s2.close()
    print("multi-size launches", stats, flush=True)
    assert stats["multi_iterations"] > 0 and stats["multi_max_grids"] >= 2
    for k in shared:
        st_alone, ra = alone[k]
        st_mix, rm = mixed[ids[k]]
        assert st_alone == 0 and st_mix == 0, k
        # bit-identical alone and in the mix
        assert np.array_equal(np.array([r["mean_stress"] for r in ra]), np.array([r["mean_stress"] for r in rm])), k
        assert [r["iters"] for r in ra] == [r["iters"] for r in rm], k
        assert [r["fp64_applications"] for r in ra] == [r["fp64_applications"] for r in rm], k
    # and identical to the single-plan path with the default tiles
    for k in ("a", "c"):
        r = shared[k]
        sol = ffth.Solver(r[0], r[2], r[3], lame=r[1], nloads=6, precision="mixed", tol=1e-8, autotune=False)
        _, rp = sol.solve_order0(np.eye(6))
        sol.close()
        assert np.array_equal(np.array([x["mean_stress"] for x in rp]),
                              np.array([x["mean_stress"] for x in alone[k][1]])), k
    for k, rid in ids.items():
        assert mixed[rid][0] == 0, k
        cm = np.array([r["mean_stress"] for r in mixed[rid][1]]).T
        assert np.abs(cm - cm.T).max() < 1e-6 * np.abs(cm).max(), k


def test_budget_admission_cancel_and_oversize():
    torch = require_gpu()
    from paper_1712_05145_amd.serving import Server
    reqs = [_req(64, 0.2, 20.0, 10 + i) for i in range(4)]
    probe = Server(64 << 20, max_running=4)
    need = probe.request_bytes((64, 64, 64), 2, 6)
    probe.close()
    budget = need + need // 2 + (1 << 20)           # room for one 64^3 request at a time
    srv = Server(budget, max_running=4)
    ids = [srv.submit(*r, np.eye(6)) for r in reqs]
    running, waiting = srv.step()
    assert running == 1 and waiting == 3
    srv.cancel(ids[3])                              # cancel a waiting request
    st, _ = srv.poll(ids[3])
    assert st == ffth.FFTH_ERR_CANCELLED
    done = _drain(srv, ids[:3])
    assert all(done[i][0] == 0 for i in ids[:3]), [done[i][0] for i in ids[:3]]
    # each request, run after a cancelled one in reused arena memory, equals the plan path
    for r, rid in zip(reqs[:3], ids[:3]):
        sol = ffth.Solver(r[0], r[2], r[3], lame=r[1], nloads=6, precision="mixed", tol=1e-8, autotune=False)
        _, rp = sol.solve_order0(np.eye(6))
        sol.close()
        assert np.array_equal(np.array([x["mean_stress"] for x in rp]),
                              np.array([x["mean_stress"] for x in done[rid][1]]))
    with pytest.raises(ffth.FFTHError) as e:       # larger than the whole arena
        srv.submit(*_req(128, 0.2, 20.0, 99), np.eye(6))
    assert e.value.status == ffth.FFTH_ERR_OOM
    srv.close()


def test_short_stream_replay_mixed_sizes():
    torch = require_gpu()
    from paper_1712_05145_amd.serving import Server, replay
    stream = M.serving_requests(count=16, rate=200.0, sizes=(32, 48, 64), seed=7)
    inputs = {}
    for r in stream:
        inputs[r["id"]] = _req(r["n"], r["fraction"], r["contrast"], r["seed"])
    srv = Server(4 << 30, max_running=16)
    records, stats = replay(srv, stream, inputs)
    srv.close()
    assert stats["requests"] == 16 and stats["failed"] == 0
    assert stats["latency_p99_ms"] >= stats["latency_p50_ms"] > 0
    print(stats)


def test_multi_size_launch_matches_oracle():
    """Requests of six grids, four of them non-cubic, on the server's four
    streams: the first two grids share their stream with the last two, and
    the inner iterations of each such pair run as one launch per pass across
    the two sizes.  Each request against the oracle's effective stiffness (CG
    to 1e-12): |dC_IJ| <= 1e-7 sqrt(C_II C_JJ)."""
    torch = require_gpu()
    from oracle import homogenization as H
    from paper_1712_05145_amd.serving import Server
    cases = []
    for shape, seed in (((16, 16, 16), 1), ((16, 24, 32), 2), ((32, 16, 24), 3), ((24, 24, 24), 4),
                        ((16, 32, 16), 5), ((24, 16, 48), 6)):
        phase = M.random_phases(shape, 3, seed)
        lame = M.lame_from_young([1.0, 8.0, 3.0], [0.3, 0.25, 0.35])
        lam0, mu0 = M.midpoint_reference(lame)
        prob = H.make_problem(phase, lam0, mu0, lame=lame)
        ceff, _, _ = H.effective_stiffness(prob, "cg", tol=1e-12)
        cases.append((phase, lame, lam0, mu0, ceff))
    srv = Server(4 << 30, max_running=8, tol=1e-10)
    ids = [srv.submit(c[0], c[1], c[2], c[3], np.eye(6)) for c in cases]
    done = _drain(srv, list(ids))
    stats = srv.stats()
    srv.close()
    print("multi-size launches", stats, flush=True)
    assert stats["multi_max_grids"] == 2
    for c, rid in zip(cases, ids):
        st, res = done[rid]
        assert st == 0
        cg = np.array([r["mean_stress"] for r in res]).T
        d = np.sqrt(np.outer(np.diag(c[4]), np.diag(c[4])))
        assert np.all(np.abs(cg - c[4]) <= 1e-7 * d), np.abs(cg - c[4]).max()


def test_multi_size_binary16_and_anisotropic_match_oracle():
    """Binary16 spectrum forced on small grids, isotropic and anisotropic
    phases: five grids on the server's four streams, so the first and the last
    share a stream and their inner iterations run as one binary16 launch per
    pass across the two sizes (for each material kind).  Every request against
    the oracle's effective stiffness (CG to 1e-12): |dC_IJ| <= 1e-7
    sqrt(C_II C_JJ)."""
    torch = require_gpu()
    from oracle import homogenization as H
    from paper_1712_05145_amd.serving import Server
    rng = np.random.default_rng(21)
    v21 = []
    for _ in range(3):
        a = rng.standard_normal((6, 6))
        c = a @ a.T + 6 * np.eye(6)
        v21.append([c[i, j] for i in range(6) for j in range(i, 6)])
    v21 = np.array(v21)
    lame = M.lame_from_young([1.0, 6.0, 2.5], [0.3, 0.25, 0.35])
    assert ffth.ffth_stiffness_contrast(voigt21=v21) <= ffth.SPECTRUM16_MAX_CONTRAST
    assert ffth.ffth_stiffness_contrast(lame=lame) <= ffth.SPECTRUM16_MAX_CONTRAST
    cases = []
    for i, shape in enumerate(((16, 16, 16), (24, 16, 16), (16, 24, 16), (16, 16, 24), (16, 32, 16))):
        phase = M.random_phases(shape, 3, 30 + i)
        lam0, mu0 = M.midpoint_reference(lame)
        ce, _, _ = H.effective_stiffness(H.make_problem(phase, lam0, mu0, lame=lame), "cg", tol=1e-12)
        cases.append((phase, lame, None, lam0, mu0, ce))
        ce, _, _ = H.effective_stiffness(H.make_problem(phase, 3.0, 3.0, voigt21=v21), "cg", tol=1e-12)
        cases.append((phase, None, v21, 3.0, 3.0, ce))
    srv = Server(4 << 30, max_running=16, tol=1e-10, spectrum16="force")
    ids = [srv.submit(c[0], c[1], c[3], c[4], np.eye(6), voigt21=c[2]) for c in cases]
    done = _drain(srv, list(ids))
    stats = srv.stats()
    srv.close()
    print("multi-size launches", stats, flush=True)
    assert stats["multi_max_grids"] == 2
    for c, rid in zip(cases, ids):
        st, res = done[rid]
        assert st == 0
        cg = np.array([r["mean_stress"] for r in res]).T
        d = np.sqrt(np.outer(np.diag(c[5]), np.diag(c[5])))
        assert np.all(np.abs(cg - c[5]) <= 1e-7 * d), np.abs(cg - c[5]).max()


def _ms(res):
    return np.array([r["mean_stress"] for r in res])


def test_cancel_running_and_close_with_rounds_in_flight():
    """Three grids on three streams, their rounds in flight: cancelling a
    running request completes its stream's round first and frees its memory;
    the other two finish bit-identical to their runs alone, and so does the
    cancelled request submitted again into the freed memory.  A server
    closed with rounds in flight drains them first, and a new server then
    computes the same results."""
    torch = require_gpu()
    from paper_1712_05145_amd.serving import Server
    reqs = {"a": _req(64, 0.25, 20.0, 41), "b": _req(32, 0.3, 30.0, 42), "c": _req(48, 0.2, 10.0, 43)}
    alone = {k: _alone(r) for k, r in reqs.items()}
    assert all(alone[k][0] == 0 for k in reqs)
    srv = Server(8 << 30, max_running=8)
    ids = {k: srv.submit(*r, np.eye(6)) for k, r in reqs.items()}
    running, waiting = srv.step()
    assert running == 3 and waiting == 0
    srv.step()
    srv.cancel(ids["a"])          # a 64^3 solve is still running after two steps
    st, _ = srv.poll(ids["a"])
    assert st == ffth.FFTH_ERR_CANCELLED
    done = _drain(srv, [ids["b"], ids["c"]])
    for k in ("b", "c"):
        st, res = done[ids[k]]
        assert st == 0, k
        assert np.array_equal(_ms(res), _ms(alone[k][1])), k
    rid = srv.submit(*reqs["a"], np.eye(6))
    st, res = _drain(srv, [rid])[rid]
    assert st == 0 and np.array_equal(_ms(res), _ms(alone["a"][1]))
    for r in reqs.values():
        srv.submit(*r, np.eye(6))
    srv.step()
    srv.step()
    srv.close()
    st, res = _alone(reqs["b"])
    assert st == 0 and np.array_equal(_ms(res), _ms(alone["b"][1]))
