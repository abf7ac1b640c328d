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


def test_alone_equals_mix_and_plan_path():
    """Request a (128^3, stiffness contrast within the binary16 limit) shares its
    grid with a request above the limit: the server runs the two in separate
    launch groups, and a's results are the same alone, in the mix and through
    the plan path."""
    torch = require_gpu()
    from paper_1712_05145_amd.serving import Server
    a = _req(128, 0.25, 20.0, 1)
    others = [_req(64, 0.3, 200.0, 2), _req(48, 0.2, 10.0, 3), _req(128, 0.35, 400.0, 4), _req(64, 0.1, 5.0, 5)]
    lim = ffth.SPECTRUM16_MAX_CONTRAST
    assert ffth.ffth_stiffness_contrast(lame=a[1]) <= lim < ffth.ffth_stiffness_contrast(lame=others[2][1])
    budget = 16 << 30
    s1 = Server(budget, max_running=8)
    ida = s1.submit(*a, np.eye(6))
    alone = _drain(s1, [ida])[ida]
    s1.close()
    s2 = Server(budget, max_running=8)
    ids = [s2.submit(*others[0], np.eye(6)), s2.submit(*others[1], np.eye(6))]
    idb = s2.submit(*a, np.eye(6))
    ids += [idb, s2.submit(*others[2], np.eye(6)), s2.submit(*others[3], np.eye(6))]
    mixed = _drain(s2, list(ids))
    s2.close()
    assert alone[0] == 0 and mixed[idb][0] == 0
    ra = np.array([r["mean_stress"] for r in alone[1]])
    rm = np.array([r["mean_stress"] for r in mixed[idb][1]])
    assert np.array_equal(ra, rm)                     # bit-identical alone and in the mix
    assert [r["iters"] for r in alone[1]] == [r["iters"] for r in mixed[idb][1]]
    # and identical to the single-plan path
    sol = ffth.Solver(a[0], a[2], a[3], lame=a[1], nloads=6, precision="mixed", tol=1e-8)
    _, rp = sol.solve_order0(np.eye(6))
    assert np.array_equal(np.array([r["mean_stress"] for r in rp]), ra)
    for rid in ids:
        assert mixed[rid][0] == 0
        c = np.array([r["mean_stress"] for r in mixed[rid][1]]).T
        assert np.abs(c - c.T).max() < 1e-6 * np.abs(c).max()


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
        sol = ffth.Solver(r[0], r[2], r[3], lame=r[1], nloads=6, precision="mixed", tol=1e-8)
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
