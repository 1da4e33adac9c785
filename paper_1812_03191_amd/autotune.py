"""Launch-shape autotuner.

The streaming y and z transport passes walk column segments of ``tile_chunk``
cells: short segments give more waves but reload more halo cells, long ones the
reverse, and the best length depends on the mesh, the storage type and how
full the GPU is.  The choice changes only the launch shape, never the results
(each face transfer is computed the same way whichever segment holds it).
``best_chunk`` times each candidate and caches the winner per (mesh,
precision, context) in a JSON file (``DFMESH_TUNE_CACHE`` or
``~/.cache/dfmesh/autotune.json``):

* batched (the default, for the engine): copies of the job advanced together
  by an engine, enough of them to fill the GPU (about 16 M cells, at most 64
  copies), as the engine's batched launches run them; the winner is the fastest
  per job-step.
* alone: a scratch run by itself; the winner is the longest segment within
  ``SLACK`` of the fastest (a lone run hides a short segment's halo rows behind
  its extra waves, which a shared GPU does not).
"""
from __future__ import annotations

import json
import os
import threading

CANDIDATES = (8, 16, 32, 64)
SLACK = float(os.environ.get("DFMESH_TUNE_SLACK", "0.15"))
_lock = threading.Lock()
_mem: dict = {}


def cache_path() -> str:
    return os.environ.get("DFMESH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dfmesh", "autotune.json"))


def key(cfg: dict, precision: int) -> str:
    # the passes of every level of a run have the shape of its level 0 (plus
    # ghosts), so one single-level timing per mesh and precision serves all
    return f"{cfg['nx']}x{cfg['ny']}x{cfg['nz']}:{'fp32' if precision else 'fp64'}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(d: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + f".{os.getpid()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def time_chunk(cfg: dict, precision: int, chunk: int, *, steps=6, warmup=2) -> float:
    """milliseconds per coarse step of a scratch run with this segment length"""
    import torch

    from ._lib import Run

    r = Run(cfg["nx"], cfg["ny"], cfg["nz"], nlevels=1, dx0=cfg["dx0"],
            gamma=cfg.get("gamma", 5.0 / 3.0), cfl=cfg.get("cfl", 0.4), precision=precision,
            seed=cfg.get("seed", 1), noise_amp=cfg.get("noise_amp", 1e-6), tile_chunk=chunk)
    r.set_perturber(cfg["GM"], cfg["eps"], cfg["L"], cfg["mach"], cfg["chi"])
    r.step(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(r.stream)
    r.step(steps)
    e1.record(r.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


BATCH_CELLS = 16 << 20
MAX_COPIES = 64


def time_chunk_batched(cfg: dict, precision: int, chunk: int, *, steps=6, warmup=2) -> float:
    """milliseconds per job-step of copies of a single-level run of this mesh
    advanced together by an engine with this segment length"""
    import torch

    from ._lib import Engine, engine_job_bytes

    one = dict(cfg, nlevels=1)
    one.pop("n1", None)
    copies = max(1, min(MAX_COPIES, -(-BATCH_CELLS // (cfg["nx"] * cfg["ny"] * cfg["nz"]))))
    eng = Engine(copies * engine_job_bytes(one, precision) + (64 << 20))
    for _ in range(copies):
        if eng.admit(one, steps + warmup, precision=precision, tile_chunk=chunk) is None:
            raise RuntimeError("autotune: engine budget too small")
    eng.step(warmup // 2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(eng.stream)
    eng.step(steps // 2)
    e1.record(eng.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (steps * copies)
    del eng
    return ms


def best_chunk(cfg: dict, precision: int, *, use_cache=True, batched=True) -> int:
    k = key(cfg, precision) + (":batched" if batched else "")
    with _lock:
        if k in _mem:
            return _mem[k]
        if use_cache:
            d = _load_cache()
            if k in d:
                _mem[k] = int(d[k]["chunk"])
                return _mem[k]
    if batched:
        times = {c: time_chunk_batched(cfg, precision, c) for c in CANDIDATES}
        best = min(CANDIDATES, key=lambda c: times[c])
    else:
        times = {c: time_chunk(cfg, precision, c) for c in CANDIDATES}
        fastest = min(times.values())
        best = max(c for c in CANDIDATES if times[c] <= (1.0 + SLACK) * fastest)
    with _lock:
        _mem[k] = best
        if use_cache:
            d = _load_cache()
            d[k] = {"chunk": best, "ms_per_step": {str(c): round(t, 4) for c, t in times.items()}}
            _store_cache(d)
    return best
