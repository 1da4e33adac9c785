"""The batched engine (df_engine_*) through the C ABI: a job run in the engine,
alone or among others of different sizes, nesting depths and precisions (the
single-level ones advancing together in one launch per stage, the nested ones
with launches of their own), gives bitwise the results of the same job stepped
eagerly; graph replays stay equal to
the eager run with other GPU work and synchronisations between them; admission
is bound by the HBM budget; completions are reported once."""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "e", "vx", "vy", "vz")


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dfm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_03191_amd as m

    return m


def _shape(cfg, name):
    e = [cfg["nx"], cfg["ny"], cfg["nz"]]
    if name != "rho" and name != "e":
        e["xyz".index(name[1])] += 1
    return (e[2], e[1], e[0])


def _eager(dfm, cfg, steps, precision, chunk=0):
    r = dfm.Run(cfg["nx"], cfg["ny"], cfg["nz"], nlevels=cfg["nlevels"], dx0=cfg["dx0"],
                seed=cfg["seed"], noise_amp=cfg["noise_amp"], precision=precision, tile_chunk=chunk)
    r.set_perturber(cfg["GM"], cfg["eps"], cfg["L"], cfg["mach"], cfg["chi"])
    r.step(steps)
    return r


def _wait_done(eng, slots, max_polls=1000):
    import torch

    seen = set()
    for _ in range(max_polls):
        seen.update(eng.poll())
        if set(slots) <= seen:
            return seen
        torch.cuda.synchronize()
    return seen


def _mix_jobs():
    return [
        (inputs.job(48, 1, 1.2, 0.01, 0.1, 1e-3, seed=41), 8),
        (dict(inputs.job(24, 1, 0.4, 0.01, 0.1, 0.0, seed=42), nx=40, ny=24, nz=18), 12),
        (inputs.job(16, 2, 0.3, 1e-3, 0.1, 1e-3, seed=43), 6),
        (inputs.job(16, 3, 0.8, 1e-3, 0.1, 5e-4, seed=44), 10),
    ]


@pytest.mark.parametrize("precision", [0, 1])
def test_engine_job_equals_eager_run(dfm, precision):
    cfg = inputs.job(32, 1, 0.7, 0.01, 0.1, 1e-3, seed=5)
    _say(f"[engine] job vs eager, precision {precision}")
    eng = dfm.Engine(1 << 30)
    s = eng.admit(cfg, 12, precision=precision)
    eng.step(6)
    assert eng.stats()["batched"] == 1  # the single-level job took the batched launches
    assert s in _wait_done(eng, [s])
    ref = _eager(dfm, cfg, 12, precision)
    for name in FIELDS:
        assert np.array_equal(eng.field(s, 0, name, _shape(cfg, name)), ref.field(0, name)), name
    assert np.array_equal(eng.force(s), ref.force())


@pytest.mark.parametrize("precision", [1, 0])
def test_engine_solo_equals_mix(dfm, precision):
    # the same job alone and among jobs of other sizes, depths and step counts
    cfg = inputs.job(32, 2, 0.5, 2e-3, 0.1, 1e-3, seed=7)
    steps = 10
    _say(f"[engine] solo vs mix, precision {precision}")
    solo = dfm.Engine(1 << 30)
    a = solo.admit(cfg, steps, precision=precision)
    solo.step(steps // 2)
    _wait_done(solo, [a])
    mix = dfm.Engine(2 << 30)
    others = [mix.admit(c, n, precision=precision) for c, n in _mix_jobs()[:2]]
    b = mix.admit(cfg, steps, precision=precision)
    others += [mix.admit(c, n, precision=precision) for c, n in _mix_jobs()[2:]]
    assert None not in others and b is not None
    mix.step(2)
    # a job admitted while the others run joins at the next step
    late = mix.admit(inputs.job(24, 1, 2.0, 0.01, 0.1, 1e-3, seed=45), 4, precision=precision)
    mix.step(steps // 2)
    _wait_done(mix, [b, late])
    for lev in range(2):
        for name in FIELDS:
            x = solo.field(a, lev, name, _shape(cfg, name))
            y = mix.field(b, lev, name, _shape(cfg, name))
            assert np.array_equal(x, y), (lev, name)
    assert np.array_equal(solo.force(a), mix.force(b))
    st = mix.stats()
    assert st["captures"] >= 2  # the set of jobs changed while running
    assert solo.stats()["batched"] == 0  # a nested job keeps launches of its own


def test_graph_replays_match_eager_between_replays(dfm):
    import torch

    cfg = inputs.job(32, 1, 0.9, 0.01, 0.1, 1e-3, seed=9)
    _say("[engine] replay-by-replay vs eager")
    eng = dfm.Engine(1 << 30)
    s = eng.admit(cfg, 40, precision=1)
    other = eng.admit(inputs.job(48, 2, 0.3, 1e-3, 0.1, 0.0, seed=10), 40, precision=1)
    ref = _eager(dfm, cfg, 0, 1)
    for r in range(5):
        eng.step(1)
        # unrelated eager work and synchronisations between replays
        x = torch.randn(1 << 20, device="cuda")
        _ = float((x * x).sum())
        torch.cuda.synchronize()
        ref.step(2)
        assert np.array_equal(eng.force(s), ref.force()), r
    assert np.array_equal(eng.field(s, 0, "rho", _shape(cfg, "rho")), ref.field(0, "rho"))
    assert other is not None


def test_engine_admission_bound_by_budget(dfm):
    cfg = inputs.job(48, 1, 0.5, 0.01, 0.1, 0.0, seed=11)
    need = dfm.engine_job_bytes(cfg, 1)
    eng = dfm.Engine(int(2.5 * need))
    a = eng.admit(cfg, 4, precision=1)
    b = eng.admit(cfg, 4, precision=1)
    c = eng.admit(cfg, 4, precision=1)
    assert a is not None and b is not None and c is None
    eng.release(a)
    c = eng.admit(cfg, 4, precision=1)
    assert c is not None
    eng.step(2)
    assert set(_wait_done(eng, [b, c])) >= {b, c}


def test_engine_completion_reported_once(dfm):
    eng = dfm.Engine(1 << 30)
    short = eng.admit(inputs.job(24, 1, 0.5, 0.01, 0.1, 0.0, seed=12), 4, precision=1)
    long_ = eng.admit(inputs.job(24, 1, 0.5, 0.01, 0.1, 0.0, seed=13), 9, precision=1)  # rounds to 10
    eng.step(2)
    got = _wait_done(eng, [short])
    assert short in got and long_ not in got
    assert eng.active()[0] == 1
    eng.step(3)
    got2 = _wait_done(eng, [long_])
    assert long_ in got2 and short not in got2
    assert eng.active()[0] == 0
    f = eng.force(long_)
    assert abs(f[3] - eng.force(short)[3] * 10 / 4) < 1e-9 * f[3]  # same dt, 10 vs 4 steps


def test_batched_sweep_subset_against_oracle(dfm):
    # the 64-job sweep, one job per mesh size (stratified subset of 4), run
    # together by the engine in FP32 and in FP64 for the sweep's 200 steps:
    # each job's force against the FP64 oracle
    from oracle.oracle import Oracle

    jobs, steps = inputs.config4()
    subset, seen = [], set()
    for c in jobs:
        if c["nx"] not in seen:
            seen.add(c["nx"])
            subset.append(c)
    _say(f"[engine] sweep subset {[c['nx'] for c in subset]} x {steps} steps vs oracle")
    want = []
    for c in subset:
        o = Oracle(c["nx"], c["ny"], c["nz"], nlevels=1, dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"],
                   seed=c["seed"], noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"], L=c["L"],
                   mach=c["mach"], chi=c["chi"])
        o.step(steps)
        want.append(o.force()[0])
    for prec, tol in ((1, 1e-4), (0, 1e-9)):
        eng = dfm.Engine(2 << 30)
        slots = [eng.admit(c, steps, precision=prec) for c in subset]
        eng.step(steps // 2)
        assert set(_wait_done(eng, slots)) >= set(slots)
        for c, s, w in zip(subset, slots, want):
            got = eng.force(s)[0]
            _say(f"[engine] n={c['nx']} mach={c['mach']:.3f} prec={prec} rel err {abs(got - w) / abs(w):.2e}")
            assert abs(got - w) <= tol * abs(w), (c["nx"], prec, got, w)


def test_release_before_poll_is_never_reported(dfm):
    # a job that finished on the device and is released before any poll
    # reported it must not be reported later, when its slot holds a new job
    import torch

    eng = dfm.Engine(1 << 30)
    a = eng.admit(inputs.job(16, 1, 0.5, 0.01, 0.1, 0.0, seed=14), 2, precision=1)
    eng.step(1)
    torch.cuda.synchronize()
    eng.release(a)
    b = eng.admit(inputs.job(16, 1, 0.5, 0.01, 0.1, 0.0, seed=15), 4, precision=1)
    assert b == a  # the lowest free slot is reused
    assert eng.poll() == []
    eng.step(2)
    got = _wait_done(eng, [b])
    assert got == {b}
    assert eng.poll() == []
    ref = _eager(dfm, inputs.job(16, 1, 0.5, 0.01, 0.1, 0.0, seed=15), 4, 1)
    assert np.array_equal(eng.force(b), ref.force())


@pytest.mark.parametrize("precision", [1, 0])
def test_engine_jobs_at_other_segment_lengths(dfm, precision):
    # jobs admitted with the column-segment lengths the autotuner chooses run
    # in one engine and give bitwise the eager run at the same length
    cases = [(inputs.job(48, 1, 1.2, 0.01, 0.1, 1e-3, seed=46), 8),
             (inputs.job(32, 2, 0.4, 2e-3, 0.1, 1e-3, seed=47), 64),
             (inputs.job(64, 1, 2.5, 0.01, 0.1, 0.0, seed=48), 16)]
    steps = 6
    _say(f"[engine] segment lengths 8, 64, 16, precision {precision}")
    eng = dfm.Engine(2 << 30)
    slots = [eng.admit(c, steps, precision=precision, tile_chunk=ch) for c, ch in cases]
    eng.step(steps // 2)
    assert set(_wait_done(eng, slots)) >= set(slots)
    for (c, ch), s in zip(cases, slots):
        ref = _eager(dfm, c, steps, precision, chunk=ch)
        for lev in range(c["nlevels"]):
            for name in FIELDS:
                assert np.array_equal(eng.field(s, lev, name, _shape(c, name)), ref.field(lev, name)), (ch, name)
        assert np.array_equal(eng.force(s), ref.force()), ch


def test_serve_results_equal_jobs_run_alone(dfm):
    # a small stream through the continuous-batching loop under a budget that
    # holds only some of the jobs at once: every job's force is bitwise that of
    # the same job run alone
    from paper_1812_03191_amd.serve import serve

    rng = np.random.default_rng(51)
    jobs = []
    for j in range(7):
        n = int(rng.choice([16, 24, 32]))
        nl = int(rng.integers(1, 3)) if n % 16 == 0 else 1
        mach = float(np.exp(rng.uniform(np.log(0.2), np.log(2.5))))
        jobs.append(inputs.job(n, nl, mach, 0.01, 0.1, 1e-3, seed=5100 + j))
    arrivals = np.cumsum(rng.exponential(0.02, size=len(jobs)))
    steps = 10
    need = max(dfm.engine_job_bytes(c, dfm.DF_FP32) for c in jobs)
    budget = int(2.2 * need)
    _say(f"[serve] {len(jobs)} jobs, budget {budget / 2**20:.1f} MiB")
    r = serve(arrivals, jobs, steps, budget_bytes=budget, precision=dfm.DF_FP32, tune=False)
    assert r["max_active"] < len(jobs)  # admission was bound by the budget
    assert r["p99_latency_s"] >= r["p50_latency_s"] > 0.0
    for j, c in enumerate(jobs):
        ref = _eager(dfm, c, steps, dfm.DF_FP32)
        assert np.array_equal(r["forces"][j], ref.force()), j
