"""Load driver for the betweenness server: replays a timed request stream
against an NkServer (requests are submitted at their arrival times from one
thread while the server's scheduler admits and runs them) and reports
latency percentiles and throughput."""
from __future__ import annotations

import time

import numpy as np

from ._lib import NkServer


def replay(server: NkServer, graph_ids, requests, timeout: float = 600.0):
    """Submits each request at its arrival time (request["t"] seconds after
    the start), then waits for all.  Returns (results, wall_seconds) with
    results[i] = (scores, latency_seconds)."""
    tickets = []
    t0 = time.perf_counter()
    for rq in requests:
        delay = rq["t"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        gid = graph_ids[rq["graph"]]
        if "sources" in rq:
            tickets.append(server.submit(gid, sources=rq["sources"], seed=rq["seed"]))
        else:
            tickets.append(server.submit(gid, eps=rq["eps"], delta=rq["delta"], seed=rq["seed"]))
    results = [server.wait(t, timeout) for t in tickets]
    return results, time.perf_counter() - t0


def latency_summary(results) -> dict:
    lat = np.array([r[1] for r in results]) * 1e3
    if lat.size == 0:
        return {"count": 0}
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max())}
