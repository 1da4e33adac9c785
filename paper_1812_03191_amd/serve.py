"""Continuous-batching job server over the engine (df_engine_*).

Jobs (independent runs of a Mach / luminosity sweep, of different mesh sizes
and nesting depths) arrive at given times.  The loop admits queued jobs in
arrival order while the engine's HBM budget and slots allow, advances every
active job together (one engine step = two coarse steps of each, captured in a
HIP graph), collects jobs as their last step completes on the device, reads
their force and frees their memory for the next admissions.  Jobs arriving
while others run join at the next engine step, so their work overlaps on the
device.  Latency of a job = completion time - arrival time.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from ._lib import DF_FP32, Engine, engine_job_bytes


def job_cell_updates(cfg: dict, steps: int) -> int:
    """active cells x (sub)steps: level l advances 2^l times per coarse step"""
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    n1 = cfg.get("n1")
    m = n1[0] * n1[1] * n1[2] if n1 else n
    return steps * (n + m * sum(2 ** l for l in range(1, cfg["nlevels"])))


def serve(arrivals, jobs, steps, *, budget_bytes, precision=DF_FP32, nstreams=4, tune=True,
          inflight=4, log=None):
    import torch

    from .autotune import best_chunk

    arrivals = np.asarray(arrivals, dtype=float)
    order = np.argsort(arrivals, kind="stable")
    chunks = {}
    for cfg in jobs:
        if engine_job_bytes(cfg, precision) > budget_bytes:
            raise ValueError("a job does not fit the HBM budget")
        # single-level jobs advance in the engine's batched launches (a full
        # GPU); nested ones launch by themselves, beside the others
        k = (cfg["nx"], cfg["ny"], cfg["nz"], cfg["nlevels"] == 1)
        if tune and k not in chunks:
            chunks[k] = best_chunk(cfg, precision, batched=k[3])
    eng = Engine(budget_bytes, nstreams=nstreams)
    stream = eng.stream
    torch.cuda.synchronize()
    queue = collections.deque()
    slot_job, admitted, done_at, forces = {}, {}, {}, {}
    events = collections.deque()
    nxt = 0
    t0 = time.perf_counter()
    max_active = 0
    while len(done_at) < len(jobs):
        now = time.perf_counter() - t0
        while nxt < len(jobs) and arrivals[order[nxt]] <= now:
            queue.append(int(order[nxt]))
            nxt += 1
        while queue:
            j = queue[0]
            cfg = jobs[j]
            k = (cfg["nx"], cfg["ny"], cfg["nz"], cfg["nlevels"] == 1)
            slot = eng.admit(cfg, steps, precision=precision, tile_chunk=chunks.get(k, 0))
            if slot is None:
                break
            queue.popleft()
            slot_job[slot] = j
            admitted[j] = time.perf_counter() - t0
        nact, _ = eng.active()
        max_active = max(max_active, nact)
        if nact:
            eng.step(1)
            ev = torch.cuda.Event()
            ev.record(stream)
            events.append(ev)
            while len(events) > inflight:
                events.popleft().synchronize()
        elif events:
            events.popleft().synchronize()
        for s in eng.poll():
            j = slot_job.pop(s)
            done_at[j] = time.perf_counter() - t0
            forces[j] = eng.force(s)
            eng.release(s)
            if log:
                log(f"[serve] job {j} done: latency {done_at[j] - arrivals[j]:.3f} s")
        if not nact and not queue and not events and nxt < len(jobs) and len(done_at) < len(jobs):
            wait = arrivals[order[nxt]] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([done_at[j] - arrivals[j] for j in range(len(jobs))])
    work = sum(job_cell_updates(c, steps) for c in jobs)
    first = float(arrivals.min())
    return {
        "jobs": len(jobs), "steps": steps, "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
        "wall_s": wall, "cell_updates": work, "cell_updates_per_s": work / (wall - first),
        "max_active": max_active, "engine": eng.stats(), "forces": forces,
        "queue_wait_s": float(np.mean([admitted[j] - arrivals[j] for j in range(len(jobs))])),
    }
