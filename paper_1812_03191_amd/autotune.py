"""Launch-shape autotuner.

The streaming y and z transport passes walk column segments of ``tile_chunk``
cells: short segments give more waves but reload more halo cells, long ones the
reverse, and the best length depends on the mesh and the storage type.  The
choice changes only the launch shape, never the results (each face transfer is
computed the same way whichever segment holds it).  ``best_chunk`` times a few
steps of a scratch run for each candidate and caches the winner per
(mesh, levels, precision) in a JSON file (``DFMESH_TUNE_CACHE`` or
``~/.cache/dfmesh/autotune.json``).  The winner is the longest segment whose
lone-run time is within ``SLACK`` of the fastest: jobs of the batching engine
share the GPU, where the halo rows a short segment recomputes cost throughput
that a lone run hides behind its extra waves.
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


def best_chunk(cfg: dict, precision: int, *, use_cache=True) -> int:
    k = key(cfg, precision)
    with _lock:
        if k in _mem:
            return _mem[k]
        if use_cache:
            d = _load_cache()
            if k in d:
                _mem[k] = int(d[k]["chunk"])
                return _mem[k]
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
