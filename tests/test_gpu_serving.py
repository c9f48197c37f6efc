"""The request loop (vts_server) on the GPU: results in a mix of concurrent
requests equal the results of each problem solved alone, admission respects
the device pool, and contexts stay inside their declared footprint."""
import numpy as np
import pytest

import workloads as W
from oracle import kkt, pbm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1904_06556_amd import serve, vts as V  # noqa: E402


def say(*a):
    print("[serving]", *a, flush=True)


def _mix():
    return [
        W.cantilever_edge(16, 8, 8, 3, vol_frac=0.3),
        W.bridge_top(16, 8, 8, 3, vol_frac=0.2, h=0.25),
        W.cantilever_edge(32, 16, 16, 4, vol_frac=0.15),
        W.bridge_top(32, 16, 16, 4, vol_frac=0.25, h=0.125),
        W.cantilever_edge(8, 4, 4, 3, vol_frac=0.4),
    ]


def test_allocated_bytes_within_footprint():
    for pr in _mix():
        for prec in (V.VTS_FP64, V.VTS_MIXED):
            say("footprint", pr.name, prec)
            ctx = V.Context.from_problem(pr, precision=prec)
            foot = V.Context.footprint_bytes(pr.nx, pr.ny, pr.nz, pr.levels, prec)
            assert 0 < ctx.allocated_bytes() <= foot
            ctx.close()


def test_mix_equals_alone():
    probs = _mix()
    alone = []
    for pr in probs:
        say("alone", pr.name)
        ctx = V.Context.from_problem(pr, precision=V.VTS_MIXED)
        r = ctx.pbm_solve()
        d = ctx.state_dict()
        alone.append((r, d["rho"].copy(), d["u"].copy()))
        ctx.close()
    feet = [V.Context.footprint_bytes(p.nx, p.ny, p.nz, p.levels, V.VTS_MIXED) for p in probs]
    # a pool that holds the two largest at once: the others wait for ranges
    pool = sorted(feet)[-1] + sorted(feet)[-2]
    say("mix: pool", pool, "footprints", feet)
    srv = V.Server(3, pool)
    recs = serve.run_stream(srv, [(0.0, p) for p in probs], precision=V.VTS_MIXED,
                            keep_fields=True)
    srv.close()
    for pr, (r, rho, u), rec in zip(probs, alone, recs):
        say("compare", pr.name, rec["status"], rec["outer"], r["outer"])
        assert rec["status"] == V.VTS_OK
        assert (rec["outer"], rec["newton"], rec["minres"]) == (r["outer"], r["newton"],
                                                                 r["minres"])
        assert rec["compliance"] == r["compliance"]
        assert np.array_equal(rec["rho"], rho) and np.array_equal(rec["u"], u)
        P = pbm.VTS(pr)
        k = kkt.kkt_residual(P.grid, P.Ke, P.f, P.V, P.rho_lo, P.rho_hi, rec["rho"], rec["u"],
                             r["alpha"])
        assert k["kkt"] <= 1e-6, (pr.name, k)
    # requests overlapped on the device while the pool allowed it
    spans = sorted((rec["t_done"] - rec["service"], rec["t_done"]) for rec in recs)
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))


def test_admission_respects_pool():
    probs = [W.cantilever_edge(32, 16, 16, 4, vol_frac=0.2 + 0.02 * k) for k in range(4)]
    foot = V.Context.footprint_bytes(32, 16, 16, 4, V.VTS_MIXED)
    srv = V.Server(4, foot + foot // 2)      # room for one request at a time
    say("admission: pool", foot + foot // 2)
    recs = serve.run_stream(srv, [(0.0, p) for p in probs], precision=V.VTS_MIXED)
    srv.close()
    spans = sorted((r["t_done"] - r["service"], r["t_done"]) for r in recs)
    assert all(r["status"] == V.VTS_OK for r in recs)
    for a, b in zip(spans, spans[1:]):
        assert b[0] >= a[1] - 1e-6              # never two admitted at once


def test_submit_rejects():
    srv = V.Server(1, 1 << 20)
    with pytest.raises(V.VtsError):
        srv.submit(W.cantilever_edge(64, 32, 32, 5))         # larger than the pool
    bad = W.cantilever_edge(8, 4, 4, 3)
    bad.V = 10 * bad.m                                       # infeasible volume
    with pytest.raises(V.VtsError):
        srv.submit(bad)
    srv.close()


def test_group_step_equals_single_steps():
    probs = _mix()[:3]
    streams = [torch.cuda.Stream() for _ in probs]
    grouped = [V.Context.from_problem(p, precision=V.VTS_MIXED, stream=s)
               for p, s in zip(probs, streams)]
    single = [V.Context.from_problem(p, precision=V.VTS_MIXED) for p in probs]
    for it in range(3):
        say("group step", it)
        gs = V.group_step(grouped)
        for k, c in enumerate(single):
            a = c.pbm_iterate()
            assert a == gs[k]
    for g, c in zip(grouped, single):
        assert np.array_equal(g.get_state(), c.get_state())
        g.close()
        c.close()


def test_fetch_before_poll():
    # a finished request may be fetched before any poll has reported it; the
    # next poll then reports only the others
    import time
    probs = [W.cantilever_edge(8, 4, 4, 3, vol_frac=0.3), W.cantilever_edge(8, 4, 4, 3, vol_frac=0.35)]
    srv = V.Server(2, 1 << 30)
    ids = [srv.submit(p, precision=V.VTS_FP64) for p in probs]
    say("fetch before poll", ids)
    t0 = time.time()
    while srv.counts()["finished"] < 2:
        assert time.time() - t0 < 60, srv.counts()
        time.sleep(0.05)
    rho, u = srv.fetch(ids[0], probs[0].m, probs[0].n_dof)
    assert np.all(np.isfinite(rho)) and np.all(np.isfinite(u))
    infos = srv.poll(timeout_s=1.0)
    assert [i["id"] for i in infos] == [ids[1]]
    with pytest.raises(V.VtsError):
        srv.fetch(ids[0], probs[0].m, probs[0].n_dof)
    srv.fetch(ids[1], probs[1].m, probs[1].n_dof)
    srv.close()


def test_same_shape_requests_share_launches_and_match_unbatched():
    # four requests of one grid (two loads, two volumes) admitted together:
    # their MINRES steps go out as shared launches, and every result is
    # bitwise the one the server gives with batching off
    probs = [W.cantilever_edge(16, 8, 8, 3, vol_frac=0.25), W.bridge_top(16, 8, 8, 3, vol_frac=0.2, h=0.25),
             W.cantilever_edge(16, 8, 8, 3, vol_frac=0.35), W.bridge_top(16, 8, 8, 3, vol_frac=0.3, h=0.25)]
    runs = {}
    for batching in (False, True):
        say("same-shape requests, batching", batching)
        srv = V.Server(4, 1 << 30, batching=batching)
        runs[batching] = serve.run_stream(srv, [(0.0, p) for p in probs], precision=V.VTS_MIXED,
                                          keep_fields=True)
        stats = srv.group_stats()
        srv.close()
        say("  group stats", stats)
        if batching:
            assert stats["solves"] > 0 and stats["max_batch"] >= 2
            assert stats["mean_batch"] > 1.0
        else:
            assert stats["launches"] == 0
    for a, b in zip(runs[False], runs[True]):
        assert a["status"] == V.VTS_OK and b["status"] == V.VTS_OK
        assert (a["outer"], a["newton"], a["minres"]) == (b["outer"], b["newton"], b["minres"])
        assert a["compliance"] == b["compliance"]
        assert np.array_equal(a["rho"], b["rho"]) and np.array_equal(a["u"], b["u"])


def test_group_step_batches_a_same_shape_pair_bitwise():
    # vts_group_step with two contexts of one shape and one of another
    probs = [W.cantilever_edge(32, 16, 16, 4, vol_frac=0.15),
             W.bridge_top(32, 16, 16, 4, vol_frac=0.25, h=0.125),
             W.cantilever_edge(16, 8, 8, 3, vol_frac=0.3)]
    streams = [torch.cuda.Stream() for _ in probs]
    grouped = [V.Context.from_problem(p, precision=V.VTS_MIXED, stream=s)
               for p, s in zip(probs, streams)]
    single = [V.Context.from_problem(p, precision=V.VTS_MIXED) for p in probs]
    for it in range(4):
        say("group step (same-shape pair)", it)
        gs = V.group_step(grouped)
        for k, c in enumerate(single):
            assert c.pbm_iterate() == gs[k]
    for g, c in zip(grouped, single):
        assert np.array_equal(g.get_state(), c.get_state())
        g.close()
        c.close()
