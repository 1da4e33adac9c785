"""Parity with the FP64 oracle on the configurations the product runs, at the
lengths the workloads use: the 128^3 single-level workload over 100 steps in
FP64 (every field within 1e-11 of its scale, the force within 1e-9) and with
FP32 departure storage (force within 1e-4, totals within 1e-6); four nested
levels of 32^3 (the nested workload at reduced size) over 20 coarse steps and
of 64^3 over 10 in both precisions; two levels of 128^3 (the nested workload's level shape)
and the nested workload itself (four levels of 128^3) over 2 coarse steps
in both precisions; and runs at every column-segment length the autotuner can
choose, bitwise equal to the default length in both precisions and within the
FP64 bar of the oracle."""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu

FIELD_NAMES = ("rho", "e", "vx", "vy", "vz")
GAMMA = 5.0 / 3.0
E0 = 1.0 / (GAMMA * (GAMMA - 1.0))
SCALE = {"rho": 1.0, "e": E0, "vx": 1.0, "vy": 1.0, "vz": 1.0}


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


def _oracle(cfg, steps):
    from oracle.oracle import Oracle

    c = cfg
    o = Oracle(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"],
               seed=c["seed"], noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"], L=c["L"], mach=c["mach"],
               chi=c["chi"])
    o.step(steps)
    res = {"force": o.force(), "totals": o.totals()[:3], "time": o.time,
           "fields": {(lev, name): o.full_field(lev, name) for lev in range(c["nlevels"]) for name in FIELD_NAMES}}
    del o
    return res


def _gpu(dfm, cfg, steps, precision, chunk=0):
    c = cfg
    g = dfm.Run(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"],
                seed=c["seed"], noise_amp=c["noise_amp"], precision=precision, tile_chunk=chunk)
    g.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
    g.step(steps)
    return g


def _check_fp64(g, ref, nlevels, what):
    errs = {}
    for lev in range(nlevels):
        for name in FIELD_NAMES:
            errs[(lev, name)] = float(np.max(np.abs(g.field(lev, name) - ref["fields"][(lev, name)]))) / SCALE[name]
    fg, fo = g.force()[:3], ref["force"]
    fe = float(np.max(np.abs(fg - fo)) / np.linalg.norm(fo))
    _say(f"[{what}] worst field error {max(errs.values()):.2e}, force error {fe:.2e}")
    assert max(errs.values()) < 1e-11, {k: v for k, v in errs.items() if v > 1e-13}
    assert fe < 1e-9, (fg, fo)
    assert abs(g.force()[3] - ref["time"]) <= 1e-12 * ref["time"]


def _check_fp32(g, ref, what):
    fg, fo = g.force()[:3], ref["force"]
    tg, to = g.totals(), ref["totals"]
    rep = {"force_rel": float(np.max(np.abs(fg - fo)) / np.linalg.norm(fo)),
           "mass_rel": float(abs(tg[0] - to[0]) / to[0]),
           "eint_rel": float(abs(tg[1] - to[1]) / to[1]),
           "ekin_rel": float(abs(tg[2] - to[2]) / to[2])}
    _say(f"[{what}] FP32 against the FP64 oracle: {rep}")
    assert rep["force_rel"] < 1e-4, rep
    assert rep["mass_rel"] < 1e-6 and rep["eint_rel"] < 1e-6 and rep["ekin_rel"] < 1e-6, rep


@pytest.fixture(scope="module")
def config2_ref():
    cfg, _ = inputs.config2()
    _say("[full parity] oracle: 128^3 x 100 steps")
    return cfg, _oracle(cfg, 100)


def test_config2_parity_100_steps_fp64(dfm, config2_ref):
    cfg, ref = config2_ref
    _say("[full parity] 128^3 FP64 x 100")
    g = _gpu(dfm, cfg, 100, dfm.DF_FP64)
    _check_fp64(g, ref, 1, "128^3 FP64")


def test_config2_100_steps_fp32_against_oracle(dfm, config2_ref):
    cfg, ref = config2_ref
    _say("[full parity] 128^3 FP32 x 100")
    g = _gpu(dfm, cfg, 100, dfm.DF_FP32)
    _check_fp32(g, ref, "128^3")


@pytest.fixture(scope="module")
def nested_ref():
    cfg, _ = inputs.config3(n=32)
    _say("[full parity] oracle: 4 levels of 32^3 x 20 coarse steps")
    return cfg, _oracle(cfg, 20)


def test_nested_four_levels_parity_fp64(dfm, nested_ref):
    cfg, ref = nested_ref
    _say("[full parity] 4 x 32^3 FP64 x 20")
    g = _gpu(dfm, cfg, 20, dfm.DF_FP64)
    _check_fp64(g, ref, 4, "4 x 32^3 FP64")


def test_nested_four_levels_fp32_against_oracle(dfm, nested_ref):
    cfg, ref = nested_ref
    _say("[full parity] 4 x 32^3 FP32 x 20")
    g = _gpu(dfm, cfg, 20, dfm.DF_FP32)
    _check_fp32(g, ref, "4 x 32^3")


@pytest.fixture(scope="module")
def nested128_ref():
    # the nested workload's level shape itself, at two levels and two coarse
    # steps: the finer level's rows with their margins are 130-148 cells, so
    # its x pass takes the wave-row form with four cells per lane (FP32) or the
    # overlapping tiles (FP64), and its walks rows longer than a wave
    cfg, _ = inputs.config3()
    cfg = dict(cfg, nlevels=2, dx0=cfg["dx0"] / 4)
    _say("[full parity] oracle: 2 levels of 128^3 x 2 coarse steps")
    return cfg, _oracle(cfg, 2)


def test_nested_128_levels_parity_fp64(dfm, nested128_ref):
    cfg, ref = nested128_ref
    _say("[full parity] 2 x 128^3 FP64 x 2")
    g = _gpu(dfm, cfg, 2, dfm.DF_FP64)
    _check_fp64(g, ref, 2, "2 x 128^3 FP64")


def test_nested_128_levels_fp32_against_oracle(dfm, nested128_ref):
    cfg, ref = nested128_ref
    _say("[full parity] 2 x 128^3 FP32 x 2")
    g = _gpu(dfm, cfg, 2, dfm.DF_FP32)
    _check_fp32(g, ref, "2 x 128^3")
    # every field of both levels against the oracle, in units of its scale:
    # FP32 holds the departures from the background, which stay below 6e-4 of
    # the scale over these two steps, so each store rounds by at most
    # 2^-24 * 6e-4; a few tens of such roundings bound the error (2.3e-9)
    worst = max(float(np.max(np.abs(g.field(lev, name) - ref["fields"][(lev, name)]))) / SCALE[name]
                for lev in range(2) for name in FIELD_NAMES)
    _say(f"[2 x 128^3] FP32 worst field error {worst:.2e}")
    assert worst < 64 * 2.0 ** -24 * 6e-4


@pytest.fixture(scope="module")
def nested64_ref():
    cfg, _ = inputs.config3(n=64)
    _say("[full parity] oracle: 4 levels of 64^3 x 10 coarse steps")
    return cfg, _oracle(cfg, 10)


def test_nested_64_levels_parity_fp64(dfm, nested64_ref):
    # finer rows of 66-84 cells with their margins: two x tiles in the fused
    # x + y pass, over ten coarse steps
    cfg, ref = nested64_ref
    _say("[full parity] 4 x 64^3 FP64 x 10")
    g = _gpu(dfm, cfg, 10, dfm.DF_FP64)
    _check_fp64(g, ref, 4, "4 x 64^3 FP64")


def test_nested_64_levels_fp32_against_oracle(dfm, nested64_ref):
    cfg, ref = nested64_ref
    _say("[full parity] 4 x 64^3 FP32 x 10")
    g = _gpu(dfm, cfg, 10, dfm.DF_FP32)
    _check_fp32(g, ref, "4 x 64^3")


@pytest.fixture(scope="module")
def nested4x128_ref():
    cfg, _ = inputs.config3()
    _say("[full parity] oracle: 4 levels of 128^3 x 2 coarse steps")
    return cfg, _oracle(cfg, 2)


def test_nested_workload_parity_fp64(dfm, nested4x128_ref):
    # the nested workload itself (4 levels of 128^3) over two coarse steps
    cfg, ref = nested4x128_ref
    _say("[full parity] 4 x 128^3 FP64 x 2")
    g = _gpu(dfm, cfg, 2, dfm.DF_FP64)
    _check_fp64(g, ref, 4, "4 x 128^3 FP64")


def test_nested_workload_fp32_against_oracle(dfm, nested4x128_ref):
    cfg, ref = nested4x128_ref
    _say("[full parity] 4 x 128^3 FP32 x 2")
    g = _gpu(dfm, cfg, 2, dfm.DF_FP32)
    _check_fp32(g, ref, "4 x 128^3")
    # FP32 holds departures from the background: each store rounds by at most
    # 2^-24 of the largest departure; a few tens of roundings bound the error
    gamma = cfg["gamma"]
    back = {"rho": 1.0, "e": 1.0 / (gamma * (gamma - 1.0)), "vx": -cfg["mach"], "vy": 0.0, "vz": 0.0}
    dep = max(float(np.max(np.abs(ref["fields"][(lev, name)] - back[name]))) / SCALE[name]
              for lev in range(4) for name in FIELD_NAMES)
    worst = max(float(np.max(np.abs(g.field(lev, name) - ref["fields"][(lev, name)]))) / SCALE[name]
                for lev in range(4) for name in FIELD_NAMES)
    _say(f"[4 x 128^3] FP32 worst field error {worst:.2e} (largest departure {dep:.2e})")
    assert worst < 64 * 2.0 ** -24 * dep


# column-segment lengths (tile_chunk) of the streaming y and z passes and of
# the fused x + y pass: the launch shape the autotuner picks
CHUNKS = (8, 16, 64)
CHUNK_CASES = [(inputs.job(64, 1, 1.1, 0.01, 0.1, 1e-3, seed=21), 10),
               (inputs.job(32, 2, 0.6, 2e-3, 0.1, 1e-3, seed=22), 4)]


@pytest.mark.parametrize("case", [0, 1])
def test_segment_length_does_not_change_results(dfm, case):
    cfg, steps = CHUNK_CASES[case]
    nl = cfg["nlevels"]
    ref = _oracle(cfg, steps)
    for prec in (dfm.DF_FP64, dfm.DF_FP32):
        base = _gpu(dfm, cfg, steps, prec)
        if prec == dfm.DF_FP64:
            _check_fp64(base, ref, nl, f"{nl} levels, default segment")
        tol = 1e-14 if prec == dfm.DF_FP64 else 1e-6
        for ch in CHUNKS:
            _say(f"[segments] {nl} levels of {cfg['nx']}^3, precision {prec}, tile_chunk {ch}")
            g = _gpu(dfm, cfg, steps, prec, chunk=ch)
            same = True
            for lev in range(nl):
                for name in FIELD_NAMES:
                    a, b = g.field(lev, name), base.field(lev, name)
                    same = same and np.array_equal(a, b)
                    assert np.max(np.abs(a - b)) <= tol * SCALE[name], (ch, lev, name)
            fa, fb = g.force(), base.force()
            same = same and np.array_equal(fa, fb)
            assert np.max(np.abs(fa[:3] - fb[:3])) <= 1e2 * tol * np.linalg.norm(fb[:3]), (ch, fa, fb)
            _say(f"[segments] tile_chunk {ch}: {'bitwise equal' if same else 'equal to rounding'} to the default")
            # a segment's first face is formed as the segment below forms it,
            # with the same roundings: the segment length changes no bit
            assert same, (prec, ch)
            if prec == dfm.DF_FP64:
                _check_fp64(g, ref, nl, f"{nl} levels, tile_chunk {ch}")
