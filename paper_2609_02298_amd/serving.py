"""Client-side drivers of the serving loop (``ib_lbm_server``).

``serve`` submits cases to a :class:`Server` at given arrival times and
collects their results; ``sequential`` runs the same cases one at a time as
plain sims (no batching) for comparison.  The request loop itself -- FIFO
admission by device footprint, continuous batching, retirement -- runs in
the library's worker thread; this module only times arrivals and summarises
latencies.
"""
from __future__ import annotations

import time

import numpy as np

from . import ib_lbm as B


def case_nodes(case: dict) -> int:
    return int(case["nx"]) * int(case["ny"])


def percentile(v, q: float) -> float:
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else float("nan")


def fifo_latencies(arrivals, service) -> list[float]:
    """Finish minus arrival of jobs served one at a time in arrival order
    with the given service times (a single FIFO server)."""
    t = 0.0
    out = []
    for a, s in zip(arrivals, service):
        t = max(t, a) + s
        out.append(t - a)
    return out


def sequential(cases, precision: int, steps=None, launch: dict | None = None,
               fields: bool = False, progress=None) -> dict:
    """Plain solves, one sim at a time on the current stream: create, add
    bodies, step, read forces (and fields), destroy.  Service time of each
    case includes its creation and teardown."""
    import torch
    out = []
    t_all = time.perf_counter()
    for i, c in enumerate(cases):
        n = int(steps[i] if steps is not None else c["steps"])
        t0 = time.perf_counter()
        sim = B.Sim(c, precision=precision)
        if launch:
            sim.set_launch(**launch)
        sim.step(n)
        sim.sync()
        bodies = [sim.forces(k, check=False) for k in range(len(c.get("bodies", [])))]
        r = dict(steps_done=sim.steps_done, bodies=bodies)
        if fields:
            r["rho"], r["ux"], r["uy"] = sim.fields()
        sim.close()
        torch.cuda.synchronize()
        r["service"] = time.perf_counter() - t0
        out.append(r)
        if progress is not None and (i + 1) % 32 == 0:
            print(f"  sequential: {i + 1}/{len(cases)} cases, {time.perf_counter() - t_all:.1f} s",
                  file=progress, flush=True)
    wall = time.perf_counter() - t_all
    nu = sum(case_nodes(c) * r["steps_done"] for c, r in zip(cases, out))
    return dict(results=out, wall=wall, node_updates=nu)


def serve(cases, precision: int, steps=None, arrivals=None, hbm_budget: int = 16 << 30,
          max_resident: int = 64, quantum: int = 256, graph_steps: int = 0,
          launch: dict | None = None, fields: bool = False, timeout: float = 600.0,
          progress=None) -> dict:
    """Submit every case at its arrival time (seconds after the start; None:
    all at once) to a fresh server and wait for all results."""
    srv = B.Server(precision=precision, hbm_budget=hbm_budget, max_resident=max_resident,
                   quantum=quantum, graph_steps=graph_steps, launch=launch)
    try:
        arr = list(arrivals) if arrivals is not None else [0.0] * len(cases)
        order = sorted(range(len(cases)), key=lambda i: arr[i])
        ids = {}
        t0 = time.perf_counter()
        for i in order:
            dt = arr[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            n = int(steps[i] if steps is not None else cases[i]["steps"])
            ids[i] = srv.submit(cases[i], n, fields=fields)
        results = [None] * len(cases)
        deadline = time.perf_counter() + timeout
        for i in range(len(cases)):
            left = deadline - time.perf_counter()
            r = srv.wait(ids[i], max(left, 0.0))
            if r is None:
                raise TimeoutError(f"request {ids[i]} of case {i} did not finish in {timeout} s")
            results[i] = r
            if progress is not None and (i + 1) % 32 == 0:
                print(f"  served: {i + 1}/{len(cases)} results, {time.perf_counter() - t0:.1f} s",
                      file=progress, flush=True)
        wall = time.perf_counter() - t0
        stats = srv.stats()
    finally:
        srv.close()
    return dict(results=results, wall=wall, stats=stats)


def summary(cases, served: dict, seq: dict, arrivals=None) -> dict:
    """Aggregate MLUPS, cases/s and latency percentiles of a served run next
    to the sequential plain solves of the same cases."""
    res = served["results"]
    ok = [r for r in res if r["status"] == 0]
    lat = [r["t_finish"] - r["t_submit"] for r in res]
    first = min(r["t_submit"] for r in res)
    last = max(r["t_finish"] for r in res)
    span = last - first
    nu = sum(case_nodes(c) * r["steps_done"] for c, r in zip(cases, res))
    service = [r["service"] for r in seq["results"]]
    arr = list(arrivals) if arrivals is not None else [0.0] * len(cases)
    seq_lat = fifo_latencies(arr, service)
    seq_span = max(a + l for a, l in zip(arr, seq_lat)) - min(arr)
    st = served["stats"]
    failures = [dict(case=c.get("name", i), status=B.STATUS.get(r["status"], r["status"]),
                     steps_done=r["steps_done"])
                for i, (c, r) in enumerate(zip(cases, res)) if r["status"] != 0]
    return {
        "cases": len(cases), "failed": len(res) - len(ok), "failures": failures[:8],
        "aggregate_mlups": round(nu / span / 1e6, 1),
        "cases_per_s": round(len(cases) / span, 3),
        "p50_latency_s": round(percentile(lat, 50), 4),
        "p99_latency_s": round(percentile(lat, 99), 4),
        "makespan_s": round(span, 3),
        "sequential": {
            "aggregate_mlups": round(seq["node_updates"] / seq_span / 1e6, 1),
            "cases_per_s": round(len(cases) / seq_span, 3),
            "p50_latency_s": round(percentile(seq_lat, 50), 4),
            "p99_latency_s": round(percentile(seq_lat, 99), 4),
            "makespan_s": round(seq_span, 3),
        },
        "peak_resident": st["peak_resident"],
        "peak_resident_gb": round(st["peak_resident_bytes"] / 2**30, 3),
        "rounds": st["rounds"],
    }
