"""Load driver for the request server: Poisson arrivals, latency percentiles.

Requests come from ``workloads.c5_request_stream`` (chains and dense systems,
s log-uniform, step counts log-uniform).  ``run_stream`` submits them to an
``osc.Server`` at their arrival times (or all at once), waits for every
result in a collector thread, and summarises the latencies the server
measured (submit to results ready) and the throughput in DOF-steps/s.
"""
from __future__ import annotations

import threading
import time
from typing import Optional

import numpy as np

from . import osc


def submit_request(srv: "osc.Server", req, method: str = "rk4", prec: str = "f32") -> int:
    w = req.system
    if req.kind == "chain":
        return srv.submit("chain", method, prec, w.m[0], w.k[0], w.dt, w.x0[0], w.v0[0], w.nsteps, w.out_stride)
    return srv.submit("dense", method, prec, w.M, w.K, w.dt, w.x0[0], w.v0[0], w.nsteps, w.out_stride)


def alone_latencies(reqs, idx, method: str = "rk4", prec: str = "f32", hbm_budget: int = 0,
                    timeout: float = 600.0) -> dict:
    """Latency of each request idx[j] served alone (one request in the server
    at a time), the reference for its slowdown in a stream."""
    out = {}
    with osc.Server(hbm_budget=hbm_budget) as srv:
        for i in idx:
            t = submit_request(srv, reqs[i], method, prec)
            out[int(i)] = srv.wait(t, timeout=timeout)["latency_s"]
    return out


def poisson_arrivals(n: int, qps: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, n))


def run_stream(reqs, arrivals: Optional[np.ndarray] = None, method: str = "rk4", prec: str = "f32",
               hbm_budget: int = 0, max_slots: int = 512, chunk_us: int = 0, timeout: float = 600.0,
               frame_jumps: bool = False) -> dict:
    """arrivals: seconds after start for each request (None: all at once).
    frame_jumps: let the server reach a dense request's frames by powers of
    its one-step matrix where that is much cheaper than stepping."""
    results = [None] * len(reqs)
    tickets = [None] * len(reqs)
    errors = []
    with osc.Server(hbm_budget=hbm_budget, max_slots=max_slots, chunk_us=chunk_us, frame_jumps=frame_jumps) as srv:
        ready = threading.Semaphore(0)

        def collect():
            for i in range(len(reqs)):
                ready.acquire()
                try:
                    results[i] = srv.wait(tickets[i], timeout=timeout)
                except osc.OscError as e:       # recorded, reported by the caller
                    errors.append((i, str(e)))
        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            if arrivals is not None:
                delay = t0 + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets[i] = submit_request(srv, r, method, prec)
            ready.release()
        th.join()
        t_end = time.perf_counter()
        stats = srv.stats()
    lat = np.array([r["latency_s"] for r in results if r is not None])
    work = sum(r.system.s * r.system.nsteps for r in reqs)
    makespan = t_end - t0
    return {
        "requests": len(reqs), "failed": len(errors), "errors": errors[:5],
        "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_latency_s": float(lat.mean()) if lat.size else None,
        "makespan_s": makespan, "dof_steps": int(work), "dof_steps_per_s": work / makespan,
        "by_frame_jumps": [i for i, r in enumerate(results) if r is not None and r.get("frame_jumps")],
        "offered_qps": (len(reqs) / arrivals[-1]) if arrivals is not None and len(arrivals) else None,
        "hbm_peak_bytes": int(stats["hbm_peak"]), "iterations": int(stats["iterations"]),
        "worker_setup_s": stats["setup_s"], "worker_iterate_s": stats["iterate_s"],
        "results": results,
    }
