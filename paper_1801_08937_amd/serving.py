"""Driving the serving engine with a request trace.

The engine itself (admission, slots, per-strategy streams, caches) is native
code behind mm_server_*; this module replays an arrival trace against it in
wall-clock time and collects latencies, and runs the same trace one request
at a time without caches for comparison.
"""
from __future__ import annotations

import time

import numpy as np


def run_trace(server, arrivals, requests, poll_sleep: float = 0.0, on_step=None):
    """Submit requests[i] = (strategy, tod, x_out, tol) at arrivals[i] seconds
    after start, stepping the server in between.  `requests` may also be a
    callable i -> request, called at the arrival (for data made on demand);
    the time stream is released once the server has admitted the request.
    on_step(elapsed_seconds) is called after every server step.
    Returns per-request info dicts (with latency) and the trace's wall time."""
    t0 = time.perf_counter()
    pending = list(range(len(arrivals)))
    ids = {}
    live = {}
    done = {}
    while pending or len(done) < len(ids):
        now = time.perf_counter() - t0
        while pending and arrivals[pending[0]] <= now:
            i = pending.pop(0)
            sid, tod, x_out, tol = requests(i) if callable(requests) else requests[i]
            ids[i] = server.submit(sid, tod, x_out, tol=tol, max_iter=2000)
            live[i] = tod
        running, queued = server.step()
        if on_step is not None:
            on_step(time.perf_counter() - t0)
        for i, rid in ids.items():
            if i in done:
                continue
            info = server.poll(rid)
            if info["state"] >= 1:
                live.pop(i, None)
            if info["state"] >= 2:
                done[i] = info
        if running == 0 and queued == 0 and pending and len(done) == len(ids):
            # idle until the next arrival
            wait = arrivals[pending[0]] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
        elif poll_sleep:
            time.sleep(poll_sleep)
    wall = time.perf_counter() - t0
    return [done[i] for i in range(len(arrivals))], wall


def latency_stats(infos, wall):
    lat = np.array([d["latency_seconds"] for d in infos])
    return {"n": int(lat.size), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "solves_per_s": float(lat.size / wall), "wall_s": float(wall),
            "converged": int(sum(d["state"] == 2 for d in infos)),
            "m2l_builds": int(sum(d["m2l_built"] for d in infos)),
            "served_with_m2l": int(sum(d.get("precond", 0) == 1 for d in infos))}
