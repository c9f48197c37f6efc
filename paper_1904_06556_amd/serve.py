"""Driver of the request loop (vts_server): replays a stream of timed VTS
requests against a Server and reports per-request latency (arrival to
result) with its percentiles.  Only submission timing and bookkeeping live
here; admission, scheduling and every solve run in the native library."""
from __future__ import annotations

import time
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import vts as V


def percentile(x: Sequence[float], q: float) -> float:
    return float(np.percentile(np.asarray(x, dtype=np.float64), q)) if len(x) else float("nan")


def run_stream(server: "V.Server", requests: Sequence[Tuple[float, object]],
               precision: int = V.VTS_MIXED, options: Optional["V.Options_t"] = None,
               on_done: Optional[Callable[[dict], None]] = None,
               keep_fields: bool = False) -> List[dict]:
    """Submits request r at its arrival time (seconds after the first call)
    and collects every result.  options: one vts_options for all requests,
    or a function of the problem that returns its options.  Returns one record per request in arrival
    order: id, arrival, status, latency (= done - arrival), service (= done -
    admit), queue (= admit - arrival), iteration counts, compliance and sizes;
    with keep_fields also the final rho and u."""
    order = sorted(range(len(requests)), key=lambda k: requests[k][0])
    t_base = server.clock() - requests[order[0]][0] if requests else 0.0
    by_id, recs = {}, [None] * len(requests)
    nxt, done = 0, 0
    while done < len(requests):
        now = server.clock() - t_base
        while nxt < len(order) and requests[order[nxt]][0] <= now:
            k = order[nxt]
            pr = requests[k][1]
            rid = server.submit(pr, precision=precision,
                                options=options(pr) if callable(options) else options)
            by_id[rid] = k
            nxt += 1
        wait = (requests[order[nxt]][0] - now) if nxt < len(order) else 1.0
        for info in server.poll(timeout_s=max(min(wait, 1.0), 0.0)):
            k = by_id[info["id"]]
            arrival = info["t_submit"]
            rec = dict(index=k, id=info["id"], status=info["status"],
                       arrival=arrival - t_base, latency=info["t_done"] - arrival,
                       service=info["t_done"] - info["t_admit"],
                       queue=info["t_admit"] - arrival, outer=info["outer"],
                       newton=info["newton"], minres=info["minres"],
                       compliance=info["compliance"], n_dof=info["n_dof"], m=info["m"],
                       footprint=info["footprint"], t_done=info["t_done"] - t_base)
            if keep_fields:
                rec["rho"], rec["u"] = server.fetch(info["id"], info["m"], info["n_dof"])
            else:
                server.fetch(info["id"], info["m"], info["n_dof"])
            recs[k] = rec
            done += 1
            if on_done is not None:
                on_done(rec)
    return recs


def summarize(recs: Sequence[dict]) -> dict:
    lat = [r["latency"] for r in recs]
    ok = [r for r in recs if r["status"] == V.VTS_OK]
    span = max(r["t_done"] for r in recs) - min(r["arrival"] for r in recs) if recs else 0.0
    return dict(n=len(recs), ok=len(ok), p50_s=percentile(lat, 50), p99_s=percentile(lat, 99),
                mean_service_s=float(np.mean([r["service"] for r in recs])) if recs else 0.0,
                mean_queue_s=float(np.mean([r["queue"] for r in recs])) if recs else 0.0,
                throughput_per_s=len(recs) / span if span > 0 else 0.0,
                dof_per_s=sum(r["n_dof"] for r in recs) / span if span > 0 else 0.0)


def time_alone(problems, precision=V.VTS_MIXED, options=None, hbm_bytes=None) -> List[dict]:
    """Each problem solved with nothing else on the device (a one-slot
    server, submitted one after the other)."""
    foot = max(V.Context.footprint_bytes(p.nx, p.ny, p.nz, p.levels, precision)
               for p in problems)
    srv = V.Server(1, hbm_bytes or foot)
    try:
        out = []
        for p in problems:
            t = time.perf_counter()
            out += run_stream(srv, [(0.0, p)], precision=precision, options=options)
            out[-1]["wall"] = time.perf_counter() - t
        return out
    finally:
        srv.close()
