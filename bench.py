#!/usr/bin/env python3
"""Throughput of the nested-mesh dynamical-friction update on one MI355X.

Workload (the configuration the headline metric is quoted on): one level of
128^3 cells in FP64, gamma 5/3, Mach 1.5, GM 0.01, chi 0.1, a luminous
perturber (L 1e-3) whose heat is released with Gaussian weights of width two
cells, seeded 1e-6 density noise.  A step is one coarse step of the whole
update: time step, kick, compression + diffusion + heat release, three
transport passes, rebuild + kick, force reduction into the force log.

Prints one JSON line: cell-updates/s (active cells x steps / wall time of the
timed steps, inputs resident in HBM), the roofline of the dominant kernel
(algorithmic bytes per launch / its average duration measured with HIP events
on the run's stream) and the FP64 CPU oracle timed on a bounded sample of the
same workload on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cell-updates/s + % HBM roofline (FP64 plain vs FP32 batched); "
          "p50/p99 job latency")
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per active cell of one launch of each kernel kind (FP64):
# the fields the kernel must read and write once each.
ALG_BYTES = {
    "kick": 8 * (5 + 3),          # read rho, e, vx, vy, vz; write vx, vy, vz
    "compress": 8 * (4 + 1),      # read e, vx, vy, vz; write e
    "kick_compress": 8 * (5 + 4),  # read rho, e, vx, vy, vz; write vx, vy, vz, e
    "diffuse_heat": 8 * (2 + 1),  # read rho, e; write e
    "pass_x": 8 * (5 + 8),        # read rho, e, vx, vy, vz; write the 8 transported
    "pass_y": 8 * (9 + 8),        # read 8 transported + vy; write 8
    "pass_z": 8 * (9 + 8),        # read 8 transported + vz; write 8
    "pass_xy": 8 * (5 + 8),       # fused x and y: read rho, e, vx, vy, vz; write the 8 transported
    "rebuild_kick": 8 * (8 + 3),  # read 8 transported; write vx, vy, vz
    # z pass fused with the rebuild and kick: read 8 transported + vz; write rho, e, vx, vy, vz
    "pass_z_finish": 8 * (9 + 5),
    # single level: the one-block kernel that sums the partials (the rebuild
    # kick forms them from the fields it already reads)
    "force": 0,
}
POST_BYTES = 8 * 5  # the separate end-of-step pass of nested runs: read rho, e, vx, vy, vz
# the method's own minimum per cell-update: read and write rho, e, vx, vy, vz once (FP64)
METHOD_BYTES_FP64 = 8 * (5 + 5)


def workload():
    from tests import inputs

    cfg, steps = inputs.config2()
    return cfg, steps


def dfk_hash() -> str:
    h = hashlib.sha256()
    for f in ("dfk.hip", "dfk.h"):
        with open(os.path.join(ROOT, "paper_1812_03191_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_config2.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != dfk_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def step_traffic_from_profiles():
    """HBM bytes of one whole single-level step (every kernel kind once) from
    the committed counter summary, if taken on the current kernel source"""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_config2.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != dfk_hash():
        return None
    # the end-of-run partials (post) are taken once per run, not per step
    return sum(v["bytes_per_launch"] for k, v in d.get("kernels", {}).items() if k != "post")


def host_threads():
    """threads the oracle may use on this host: the CPUs this process may run
    on, capped by OMP_NUM_THREADS when it is set (the host's share of cores)"""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return (min(avail, cap) if cap > 0 else avail), avail


def cpu_baseline(cfg, budget_s=12.0):
    """the FP64 oracle on the host: a bounded number of coarse steps of the
    same 128^3 workload, with all OpenMP threads and with one thread"""
    nthreads, avail = host_threads()
    omp_env = os.environ.get("OMP_NUM_THREADS")
    from oracle.oracle import Oracle

    cells = cfg["nx"] * cfg["ny"] * cfg["nz"]

    def rate(threads, budget):
        o = Oracle(cfg["nx"], cfg["ny"], cfg["nz"], nlevels=cfg["nlevels"], dx0=cfg["dx0"],
                   gamma=cfg["gamma"], cfl=cfg["cfl"], seed=cfg["seed"], noise_amp=cfg["noise_amp"],
                   GM=cfg["GM"], eps=cfg["eps"], L=cfg["L"], mach=cfg["mach"], chi=cfg["chi"],
                   threads=threads)
        t0 = time.perf_counter()
        o.step(1)
        t1 = time.perf_counter() - t0
        n = max(1, min(60, int(budget / max(t1, 1e-3))))
        t0 = time.perf_counter()
        o.step(n)
        el = time.perf_counter() - t0
        return cells * n / el, n, el

    v, n, el = rate(nthreads, budget_s)
    v1, n1, el1 = rate(1, budget_s / 2)
    return {"value": v, "unit": "cell-updates/s", "cores": nthreads, "kind": "oracle",
            "sample": f"128^3 single level FP64, {n} coarse steps after one untimed step "
                      f"({el:.1f} s, OpenMP threads={nthreads})",
            "value_1thread": v1,
            "sample_1thread": f"{n1} coarse steps after one untimed step ({el1:.1f} s, 1 thread)",
            "host": {"nproc": os.cpu_count(), "cpus_allowed": avail,
                     "omp_num_threads": omp_env,
                     "build": "gcc -O3 -march=x86-64-v3 -ffp-contract=off -fopenmp"}}


def fp32_single(cfg, K, W):
    """the same 128^3 workload with FP32 departure storage (single run)"""
    import torch

    import paper_1812_03191_amd as dfm

    run = dfm.Run(cfg["nx"], cfg["ny"], cfg["nz"], nlevels=1, dx0=cfg["dx0"], seed=cfg["seed"],
                  noise_amp=cfg["noise_amp"], precision=dfm.DF_FP32)
    run.set_perturber(cfg["GM"], cfg["eps"], cfg["L"], cfg["mach"], cfg["chi"])
    run.step(W)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(run.stream)
    run.step(K)
    e1.record(run.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = cfg["nx"] * cfg["ny"] * cfg["nz"]
    return {"cell_updates_per_s": cells * K / (ms / 1e3), "ms_per_step": ms / K, "force": run.force()[:3].tolist()}


def nested(steps=None, warm=2):
    """4 levels of 128^3 (Mach 0.3, GM 1e-3, chi 0.1, L 1e-3, 100 coarse
    steps, seed 3) in FP64 and with FP32 departures: cell-updates/s over all
    levels (level l advances 2^l sub-steps per coarse step) and the FP32
    force error against the FP64 run"""
    import numpy as np
    import torch

    import paper_1812_03191_amd as dfm
    from tests import inputs

    cfg, K = inputs.config3()
    K = steps or K
    cells = cfg["nx"] * cfg["ny"] * cfg["nz"] * sum(2 ** l for l in range(cfg["nlevels"]))
    out = {"workload": f"4 levels of 128^3, Mach 0.3, GM 1e-3, chi 0.1, L 1e-3, {K} coarse steps, seed 3"}
    forces = {}
    for name, prec in (("fp64", dfm.DF_FP64), ("fp32", dfm.DF_FP32)):
        run = dfm.Run(cfg["nx"], cfg["ny"], cfg["nz"], nlevels=cfg["nlevels"], dx0=cfg["dx0"],
                      seed=cfg["seed"], noise_amp=cfg["noise_amp"], precision=prec)
        run.set_perturber(cfg["GM"], cfg["eps"], cfg["L"], cfg["mach"], cfg["chi"])
        run.step(warm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(run.stream)
        run.step(K)
        e1.record(run.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        forces[name] = run.force()
        out[name] = {"cell_updates_per_s": cells * K / (ms / 1e3), "ms_per_coarse_step": ms / K}
        print(f"[bench] nested {name}: {K} coarse steps, {ms / K:.3f} ms each", file=sys.stderr, flush=True)
        del run
        torch.cuda.empty_cache()
    f64, f32 = forces["fp64"], forces["fp32"]
    out["fp32_force_rel_err_vs_fp64"] = float(abs(f32[0] - f64[0]) / abs(f64[0]))
    out["cell_updates_per_coarse_step"] = cells
    # against the FP64 oracle at reduced size: the same nesting with 32^3 levels, 20 coarse steps
    from oracle.oracle import Oracle

    small, Ks = inputs.config3(n=32)[0], 20
    c = small
    o = Oracle(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"],
               seed=c["seed"], noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"], L=c["L"], mach=c["mach"],
               chi=c["chi"], threads=host_threads()[0])
    o.step(Ks)
    fo = o.force()
    rel = {}
    for name, prec in (("fp64", dfm.DF_FP64), ("fp32", dfm.DF_FP32)):
        run = dfm.Run(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], seed=c["seed"],
                      noise_amp=c["noise_amp"], precision=prec)
        run.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
        run.step(Ks)
        rel[name] = float(np.max(np.abs(run.force()[:3] - fo)) / np.linalg.norm(fo))
    out["force_rel_err_vs_oracle_4x32cube_20_steps"] = rel
    return out


def batched_sweep(warm=2):
    """64 independent single-level runs (edges 48-96, Mach 0.1-3, L 0 or 1e-3),
    200 coarse steps each, FP32 departures, advanced together by the engine
    (one HIP graph replay = 2 coarse steps of every job); the same sweep in
    FP64 gives each job's force error of the FP32 storage."""
    import numpy as np
    import torch

    import paper_1812_03191_amd as dfm
    from paper_1812_03191_amd.autotune import best_chunk
    from tests import inputs

    jobs, steps = inputs.config4()
    res = {}
    forces = {}
    for prec, name in ((dfm.DF_FP32, "fp32"), (dfm.DF_FP64, "fp64")):
        chunks = {}
        for c in jobs:
            k = (c["nx"], c["ny"], c["nz"])
            if k not in chunks:
                chunks[k] = best_chunk(c, prec)
        budget = sum(dfm.engine_job_bytes(c, prec) for c in jobs) + (64 << 20)
        eng = dfm.Engine(budget, nstreams=4)
        slots = [eng.admit(c, steps + 2 * warm, precision=prec, tile_chunk=chunks[(c["nx"], c["ny"], c["nz"])])
                 for c in jobs]
        assert None not in slots
        eng.step(warm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(eng.stream)
        eng.step(steps // 2)
        e1.record(eng.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        cells = sum(c["nx"] * c["ny"] * c["nz"] for c in jobs)
        forces[name] = np.array([eng.force(s)[0] for s in slots])
        res[name] = {"cell_updates_per_s": cells * steps / (ms / 1e3), "ms_per_coarse_step": ms / steps,
                     "cells_per_coarse_step": cells, "jobs": len(jobs), "steps_each": steps,
                     "engine": eng.stats(), "tile_chunks": {f"{k[0]}": v for k, v in chunks.items()}}
        del eng
    rel = np.abs(forces["fp32"] - forces["fp64"]) / np.abs(forces["fp64"])
    res["fp32"]["force_rel_err_vs_fp64"] = {"max": float(rel.max()), "median": float(np.median(rel))}
    # against the FP64 oracle: one job per mesh size (a stratified subset)
    from oracle.oracle import Oracle

    sub, seen = [], set()
    for j, c in enumerate(jobs):
        if c["nx"] not in seen:
            seen.add(c["nx"])
            sub.append(j)
    errs = {"fp32": [], "fp64": []}
    for j in sub:
        c = jobs[j]
        o = Oracle(c["nx"], c["ny"], c["nz"], nlevels=1, dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"],
                   seed=c["seed"], noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"], L=c["L"], mach=c["mach"],
                   chi=c["chi"], threads=host_threads()[0])
        o.step(steps + 2 * warm)
        fo = o.force()[0]
        for name in errs:
            errs[name].append(abs(forces[name][j] - fo) / abs(fo))
    for name in errs:
        res[name]["force_rel_err_vs_oracle"] = {
            "jobs": [f"{jobs[j]['nx']}^3 Mach {jobs[j]['mach']:.3f}" for j in sub],
            "max": float(max(errs[name])), "per_job": [float(x) for x in errs[name]]}
    return res


def serving(njobs, budget_gb=8.0):
    """Poisson arrivals at 20 jobs/s of runs with edges 32-128 and 1-3 levels,
    300 coarse steps each, FP32 departures, continuous batching under an HBM
    budget; p50/p99 latency from arrival to completion."""
    import paper_1812_03191_amd as dfm
    from paper_1812_03191_amd.serve import serve
    from tests import inputs

    t, jobs, steps = inputs.config5()
    t, jobs = t[:njobs], jobs[:njobs]
    r = serve(t - t[0], jobs, steps, budget_bytes=int(budget_gb * (1 << 30)), precision=dfm.DF_FP32)
    r.pop("forces")
    r["budget_gb"] = budget_gb
    r["arrival_rate_per_s"] = 20.0
    return r


def copy_probe(nbytes=1 << 30):
    """the library's plain copy kernel on 1 GiB, for scaling the byte counters"""
    import torch

    import paper_1812_03191_amd as dfm

    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dfm.stream_copy(dst, src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": nbytes, "launches": 3}), file=sys.stderr)


def attainable_bandwidth(nbytes=1 << 30, reps=10):
    """GB/s (read + write) of the library's plain copy kernel over 1 GiB"""
    import torch

    import paper_1812_03191_amd as dfm

    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dfm.stream_copy(dst, src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dfm.stream_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms / 1e3) / 1e9


# kernel kind of each kernel name in a counter file (FP64 and FP32 alike):
# every listed substring must occur in the demangled name
PMC_KINDS = ((("k_kick0p<", ", false, true, false, false>"), "kick"), (("k_kick<", ", false, true>"), "kick"),
             (("k_kick0p<", ", false, true, false, true>"), "kick_compress"),
             (("k_kick0p<", ", true, true, "), "rebuild_kick"), (("k_kick<", ", true, true>"), "rebuild_kick"),
             (("k_compress",), "compress"), (("k_diffuse_heat",), "diffuse_heat"),
             (("k_xrow<",), "pass_x"), (("k_xpass<",), "pass_x"),
             (("k_march<double, 1,",), "pass_y"), (("k_march<float, 1,",), "pass_y"),
             (("k_march<double, 2,",), "pass_z"), (("k_march<float, 2,",), "pass_z"),
             (("k_xyshared<",), "pass_xy"), (("k_zfinish<",), "pass_z_finish"),
             (("k_step_final",), "force"), (("k_post<",), "post"))


def summarize_pmc(fetch_csv: str, write_csv: str, precision: str = "fp64") -> None:
    """HBM bytes per launch of each kernel kind from a FETCH_SIZE and a
    WRITE_SIZE pass of rocprofv3 over `bench.py ... --copy-probe`.  Both
    counters read in KiB per dispatch; each is scaled by what it reads for the
    1 GiB plain copies of the probe.  Writes profiles/pmc_traffic_config2.json
    (tagged with the kernel source hash) and prints a markdown table."""
    import collections
    import csv

    def load(path):
        rows = collections.defaultdict(list)
        probe = []
        for r in csv.DictReader(open(path)):
            n, v, g = r["Kernel_Name"], float(r["Counter_Value"]), int(r["Grid_Size"])
            if "k_copy16" in n:
                probe.append((g, v))
            rows[n].append(v)
        gmax = max(g for g, _ in probe)
        pv = [v for g, v in probe if g == gmax]
        return rows, (1 << 20) / (sum(pv) / len(pv))

    F, kf = load(fetch_csv)
    W, kw = load(write_csv)
    kinds = collections.defaultdict(lambda: [0.0, 0.0])
    for n in F:
        for subs, kind in PMC_KINDS:
            if all(x in n for x in subs):
                # per step: mean per dispatch, kernels of one kind summed
                kinds[kind][0] += sum(F[n]) / len(F[n]) * kf * 1024
                kinds[kind][1] += (sum(W[n]) / len(W[n]) * kw * 1024) if n in W else 0.0
                break
    out = {"source_hash": dfk_hash(), "fetch_scale": round(kf, 4), "write_scale": round(kw, 4),
           "workload": "128^3 single level FP64 (the bench workload)",
           "kernels": {k: {"fetch_bytes": int(f), "write_bytes": int(w), "bytes_per_launch": int(f + w)}
                       for k, (f, w) in sorted(kinds.items())}}
    if precision == "fp64":  # the bench line reads the FP64 figures
        with open(os.path.join(ROOT, "profiles", "pmc_traffic_config2.json"), "w") as fh:
            json.dump(out, fh, indent=1)
    esz = 4 if precision == "fp32" else 8
    cells = workload()[0]["nx"] * workload()[0]["ny"] * workload()[0]["nz"]
    print(f"scale factors: FETCH_SIZE x{kf:.3f}, WRITE_SIZE x{kw:.3f} (1 GiB copy probe)\n")
    print("| kind | fetch MiB | write MiB | total MiB | algorithmic MiB |")
    print("|---|---:|---:|---:|---:|")
    for k, (f, w) in sorted(kinds.items()):
        alg = (POST_BYTES if k == "post" else ALG_BYTES.get(k, 0)) * cells / 2**20 * esz / 8
        print(f"| {k} | {f / 2**20:.1f} | {w / 2**20:.1f} | {(f + w) / 2**20:.1f} | {alg:.1f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--device-warmup-ms", type=float, default=100.0,
                    help="run the workload this long before the warmup steps (GPU clock ramp; 0: off)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--nested-steps", type=int, default=None,
                    help="coarse steps of the nested leg (default 100; fewer under a counter profiler)")
    ap.add_argument("--no-batched", action="store_true", help="run none of the extra legs")
    ap.add_argument("--legs", default="fp32,batched,nested",
                    help="extra legs to run: any of fp32, batched, nested (comma separated)")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="storage of the timed 128^3 run (fp64 is the headline line; fp32 for profiling)")
    ap.add_argument("--serve-jobs", type=int, default=400,
                    help="jobs of the served workload to run (400 is the whole stream; 0 skips)")
    ap.add_argument("--separate-launches", action="store_true",
                    help="time the 128^3 run with every stage a launch of its own (no kernel fusion)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/pmc_traffic_config2.json from two counter passes and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, precision=args.precision)
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent runs of a sweep go to separate GPUs as separate processes)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1812_03191_amd as dfm

    cfg, default_steps = workload()
    K = args.steps if args.steps is not None else default_steps
    W = args.warmup
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()

    fp32 = args.precision == "fp32"
    esz = 4 if fp32 else 8
    run = dfm.Run(cfg["nx"], cfg["ny"], cfg["nz"], nlevels=cfg["nlevels"], dx0=cfg["dx0"],
                  gamma=cfg["gamma"], cfl=cfg["cfl"], seed=cfg["seed"], noise_amp=cfg["noise_amp"],
                  precision=dfm.DF_FP32 if fp32 else dfm.DF_FP64)
    run.set_perturber(cfg["GM"], cfg["eps"], cfg["L"], cfg["mach"], cfg["chi"])
    if args.separate_launches:
        run.set_kick_fusion(False)
        run.set_transport_fusion(False)
        run.set_finish_fusion(False)
    stream = run.stream
    # a fresh process runs its first ~100 steps about 15 % slower while the
    # GPU's clocks come up: run the workload for DEVICE_WARMUP_MS before the W
    # warmup steps (reported as device_warmup_steps), so that the K timed
    # steps see the steady state a 500-step run has
    dev_warm = 0
    if args.device_warmup_ms > 0:
        t_end = time.perf_counter() + args.device_warmup_ms / 1e3
        while time.perf_counter() < t_end and dev_warm < 2000:
            run.step(10)
            torch.cuda.synchronize()
            dev_warm += 10
    print(f"[bench] 128^3 {args.precision.upper()}: device warmup {dev_warm} steps, warmup {W}, timed {K}",
          file=sys.stderr, flush=True)
    run.step(W)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    run.step(K)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    cells = cfg["nx"] * cfg["ny"] * cfg["nz"]
    value = cells * K / (ms / 1e3)
    F = run.force()
    print(f"[bench] {ms / K:.4f} ms/step, {value:.4e} cell-updates/s", file=sys.stderr, flush=True)

    roof = None
    kern = {}
    if not args.no_kernel_timing:
        # the same K steps again, with HIP events around every launch on the run's stream
        launches = 16 * K
        dfm.timing_enable(run.handle, launches)
        run.step(K)
        kern = dfm.timing_read(run.handle)
        dfm.timing_enable(run.handle, 0)
        busy = {k: v for k, v in kern.items() if v[1] > 0 and ALG_BYTES.get(k, 0) > 0}
        # the dominant kernel: the longest launch of a step
        dom = max(busy, key=lambda k: busy[k][0] / busy[k][1])
        avg_ms = busy[dom][0] / busy[dom][1]
        # the method's algorithmic bytes per cell-update (read and write the
        # five state fields once: 80 B in FP64, 40 B in FP32) times the active
        # cells one launch advances
        per_launch = METHOD_BYTES_FP64 * cells * esz // 8
        achieved = per_launch / (avg_ms / 1e3) / 1e9
        traffic = None if fp32 else traffic_from_profiles(dom)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "avg_launch_us": round(avg_ms * 1e3, 2), "alg_bytes_per_launch": per_launch,
                "alg_bytes_basis": f"{METHOD_BYTES_FP64 * esz // 8} B per cell-update x {cells} cells"}
        att = attainable_bandwidth()
        roof["attainable"] = round(att, 1)
        roof["frac_of_attainable"] = round(achieved / att, 4)
        # the kernel's own fields read and written once each, over its duration
        own = ALG_BYTES[dom] * cells * esz // 8
        roof["kernel_alg_frac"] = round(own / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        if traffic:
            # measured DRAM bytes of the same kernel over its duration
            roof["traffic_frac"] = round(traffic / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
            roof["traffic_over_alg"] = round(traffic / per_launch, 3)
        step_traffic = None if fp32 else step_traffic_from_profiles()
        if step_traffic:
            roof["step_traffic_bytes"] = step_traffic
            roof["step_traffic_over_alg"] = round(step_traffic / per_launch, 3)
        # every kind's algorithmic bandwidth and its fraction of the HBM peak
        kern = {k: {"ms_total": round(v[0], 3), "launches": v[1],
                    "avg_us": round(1e3 * v[0] / v[1], 2) if v[1] else None,
                    "alg_GBs": round(ALG_BYTES[k] * cells * esz // 8 / (v[0] / v[1] / 1e3) / 1e9, 1)
                    if ALG_BYTES.get(k) else None,
                    "hbm_frac": round(ALG_BYTES[k] * cells * esz // 8 / (v[0] / v[1] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                    if ALG_BYTES.get(k) else None} for k, v in kern.items() if v[1]}

    extra = {}
    legs = set() if args.no_batched else set(x.strip() for x in args.legs.split(",") if x.strip())
    if "fp32" in legs:
        print("[bench] FP32 single run", file=sys.stderr, flush=True)
        extra["fp32_single"] = fp32_single(cfg, K, W)
    if "batched" in legs:
        print("[bench] batched sweep (64 jobs, FP32 and FP64)", file=sys.stderr, flush=True)
        extra["batched"] = batched_sweep()
    if "nested" in legs:
        print("[bench] nested 4 x 128^3 (FP64 and FP32)", file=sys.stderr, flush=True)
        extra["nested"] = nested(args.nested_steps)
    if args.serve_jobs > 0:
        print(f"[bench] serving {args.serve_jobs} jobs", file=sys.stderr, flush=True)
        extra["serving"] = serving(args.serve_jobs)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg)

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K,
        "warmup": W, "device_warmup_steps": dev_warm, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if fp32 else "f64", "data": "synthetic",
        "config": {"workload": f"128^3 single level {args.precision.upper()}, Mach 1.5, GM 0.01, chi 0.1, "
                               "L 1e-3, Gaussian heat width 2 cells, seed 2 (500-step run)",
                   "cells": cells, "precision": args.precision,
                   "launches": "separate" if args.separate_launches else "fused"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "force": {"Fx": F[0], "Fy": F[1], "Fz": F[2], "t": F[3]},
        "kernels": kern,
        # the whole step against the method's own minimum (read and write the 5
        # state fields once per cell-update) at the HBM peak
        "alg_efficiency": round(10.0 * esz * value / (HBM_PEAK_GBS * 1e9), 4),
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
