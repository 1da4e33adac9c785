"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle on the
same seeded inputs.  Tolerances: after the FP64 steps every field of every
level agrees within 1e-11 of its scale (rho0, e0, c_s) and the force within
1e-9 of its norm; single stages agree within 1e-13."""
import math
import os
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


def _pair(dfm, cfg, *, gf=0):
    from oracle.oracle import Oracle

    c = dict(cfg)
    o = Oracle(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"],
               cfl=c["cfl"], seed=c["seed"], noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"],
               L=c["L"], mach=c["mach"], chi=c["chi"], gf=gf or 10)
    g = dfm.Run(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"],
                cfl=c["cfl"], seed=c["seed"], noise_amp=c["noise_amp"], ghost_fine=gf)
    g.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
    return o, g


def _field_errors(o, g, nlevels):
    errs = {}
    for lev in range(nlevels):
        for name in FIELD_NAMES:
            a = g.field(lev, name)
            b = o.full_field(lev, name)
            assert a.shape == b.shape, (name, a.shape, b.shape)
            errs[(lev, name)] = float(np.max(np.abs(a - b))) / SCALE[name]
    return errs


def _force_err(o, g):
    fg = g.force()[:3]
    fo = o.force()
    return float(np.max(np.abs(fg - fo)) / max(np.linalg.norm(fo), 1e-300)), fg, fo


# ------------------------------------------------------------------ stages

def _random_pair(dfm, n, seed, *, mach=0.5, GM=0.01, eps=0.05, L=2e-3, chi=0.1):
    from oracle.oracle import Oracle

    nx, ny, nz = n
    kw = dict(dx0=0.05, GM=GM, eps=eps, L=L, mach=mach, chi=chi, noise_amp=0.0)
    o = Oracle(nx, ny, nz, **kw)
    g = dfm.Run(nx, ny, nz, dx0=0.05, noise_amp=0.0)
    g.set_perturber(GM, eps, L, mach, chi)
    st = inputs.random_state((nz, ny, nx), seed, mach=mach, e0=E0)
    rng = np.random.default_rng(seed + 1)
    for name in FIELD_NAMES:
        shp = g.shape(name)
        if name in ("rho", "e"):
            arr = st[name]
        else:
            base = -mach if name == "vx" else 0.0
            arr = base + 1e-3 * rng.uniform(-1, 1, size=shp)
            if name == "vx":
                arr[:, :, -1] = -mach  # the injection face carries the wind
        g.set_field(0, name, arr)
        o.set_full_field(0, name, arr)
    return o, g


STAGE_CASES = [("kick", 2e-3), ("compress", 2e-3), ("diffuse", 1e-3), ("heat", 1e-3),
               ("transport", 2e-3), ("sources", 1e-3), ("level_step", 2e-3)]


@pytest.mark.parametrize("stage,dt", STAGE_CASES)
@pytest.mark.parametrize("n", [(16, 16, 16), (20, 12, 18)])
def test_stage_parity(dfm, stage, dt, n):
    _say(f"[stage parity] {stage} n={n}")
    o, g = _random_pair(dfm, n, seed=17)
    o.stage(stage, dt)
    g.stage(stage, dt)
    errs = _field_errors(o, g, 1)
    worst = max(errs.values())
    assert worst < 1e-13, {k: v for k, v in errs.items() if v > 1e-14}


# The x pass takes one of several launch forms by row length on level 0:
# whole rows per wave with 1, 2 or 4 cells per lane (a row exactly filling the
# wave, a partly filled one), and the overlapping-tile form otherwise.
XROW_SHAPES = [(64, 8, 6), (128, 6, 8), (96, 6, 6), (200, 6, 4), (130, 6, 4), (256, 4, 4)]


@pytest.mark.parametrize("n", XROW_SHAPES)
@pytest.mark.parametrize("stage,dt", [("transport", 2e-3), ("level_step", 2e-3)])
def test_x_pass_launch_forms(dfm, stage, dt, n):
    _say(f"[x pass forms] {stage} n={n}")
    o, g = _random_pair(dfm, n, seed=29)
    o.stage(stage, dt)
    g.stage(stage, dt)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 1e-13, {k: v for k, v in errs.items() if v > 1e-14}


# Fused x and y passes against separate ones: one wave per row (32, 64 cells),
# two cells per lane with every lane live (128) or some lanes past the row end
# (96), y extents of one segment and of several with a ragged last one (40).
FUSED_SHAPES = [(32, 16, 8), (64, 12, 6), (96, 10, 6), (128, 40, 6), (64, 18, 4), (128, 34, 2), (64, 2, 4),
                (128, 4, 2)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", FUSED_SHAPES)
def test_fused_xy_equals_separate_passes(dfm, n, prec):
    _say(f"[fused xy] n={n} {prec}")
    nx, ny, nz = n
    p = dfm.DF_FP32 if prec == "fp32" else dfm.DF_FP64
    runs = []
    for fuse in (False, True):
        g = dfm.Run(nx, ny, nz, dx0=0.05, seed=31, noise_amp=1e-3, precision=p)
        g.set_perturber(0.01, 0.05, 2e-3, 1.3, 0.1)
        g.set_transport_fusion(fuse)
        g.step(6)
        runs.append(g)
    # the same operations in the same order; only the pairing of a product
    # and a sum into one fused multiply-add may differ between the kernels
    tol = 1e-6 if prec == "fp32" else 1e-14
    for name in FIELD_NAMES:
        a, b = runs[0].field(0, name), runs[1].field(0, name)
        assert np.max(np.abs(a - b)) <= tol * SCALE[name], (name, float(np.max(np.abs(a - b))))
    fa, fb = runs[0].force(), runs[1].force()
    assert np.max(np.abs(fa[:3] - fb[:3])) <= 1e2 * tol * np.linalg.norm(fa[:3]), (fa, fb)
    assert fa[3] == fb[3]


# Fused x and y passes of the finer levels, and of level 0 under them (with
# flux matching on their frontier; rows of 16 to 128 cells), against separate
# ones: finer rows (with their margins) in one 64-lane tile (16^3 levels), two (64^3) and three
# (128^3 with one finer level, both sub-steps' margins), y extents of one
# 32-row segment and of several, a middle level taking a finer level's
# frontier transfers, the quadrant's finest level, and supersonic runs with
# the artificial viscosity.  Rows whose last cells take half-wave tiles (FP64): 18
# and 26 cells (16^3), 76 and 66 (64^3), 140 and 130 (128^3), 62 (48^3 with
# the viscosity), and 63 over an odd number of planes (the middle level of the
# last case but one, whose last half-wave tile has no second plane); level 0
# with two cells per lane on rows that fill part of the wave (96 cells).
FINE_XY_CASES = [((16, 16, 16), 3, False, 4, 0.0), ((64, 64, 64), 2, False, 3, 0.0),
                 ((32, 32, 32), 3, False, 2, 0.0), ((128, 128, 128), 2, False, 1, 0.0),
                 ((32, 16, 16), 2, True, 3, 0.0), ((48, 48, 48), 2, False, 3, 2.0),
                 ((48, 48, 48), 3, False, 2, 2.0), ((96, 80, 64), 2, False, 2, 0.0)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(FINE_XY_CASES)))
def test_fused_xy_fine_levels_equal_separate_passes(dfm, case, prec):
    # (the last case: Mach 2 with the artificial viscosity, one more cell of margin)
    (nx, ny, nz), nl, quad, steps, visc = FINE_XY_CASES[case]
    _say(f"[fused xy fine] {nx}x{ny}x{nz}, {nl} levels, quadrant {quad}, viscosity {visc}, {prec}")
    p = dfm.DF_FP32 if prec == "fp32" else dfm.DF_FP64
    runs = []
    for fuse in (False, True):
        g = dfm.Run(nx, ny, nz, nlevels=nl, dx0=0.16, seed=33, noise_amp=1e-3, precision=p, quadrant=quad)
        if quad:
            g.set_boundaries(1)
        if visc:
            g.set_viscosity(visc)
        g.set_perturber(0.01, 0.05, 2e-3, 2.0 if visc else 0.9, 0.1)
        g.set_transport_fusion(fuse)
        g.step(steps)
        runs.append(g)
    tol = 1e-6 if prec == "fp32" else 1e-14
    for lev in range(nl):
        for name in FIELD_NAMES:
            a, b = runs[0].field(lev, name), runs[1].field(lev, name)
            assert np.max(np.abs(a - b)) <= tol * SCALE[name], (lev, name, float(np.max(np.abs(a - b))))
    fa, fb = runs[0].force(), runs[1].force()
    assert np.max(np.abs(fa[:3] - fb[:3])) <= 1e2 * tol * np.linalg.norm(fa[:3]), (fa, fb)
    assert fa[3] == fb[3]


# (in FP32 the finer levels of the nested cases take the fused launch as well)
KC_CASES = [((32, 16, 8), 1, 0), ((64, 12, 6), 1, 1), ((128, 20, 6), 1, 0), ((16, 16, 16), 2, 0),
            ((16, 16, 16), 3, 1), ((16, 2, 4), 1, 0), ((16, 2, 4), 1, 1), ((8, 4, 2), 1, 1),
            ((24, 24, 24), 4, 0), ((32, 16, 24), 2, 1)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,nl,bcmode", KC_CASES)
def test_fused_kick_compress_equals_separate(dfm, n, nl, bcmode, prec):
    _say(f"[fused kick+compress] n={n} levels={nl} bc={bcmode} {prec}")
    nx, ny, nz = n
    p = dfm.DF_FP32 if prec == "fp32" else dfm.DF_FP64
    runs = []
    for fuse in (False, True):
        g = dfm.Run(nx, ny, nz, nlevels=nl, dx0=0.05 if nl == 1 else 0.16, seed=37, noise_amp=1e-3, precision=p)
        g.set_perturber(0.01, 0.05, 2e-3, 1.3, 0.1)
        g.set_boundaries(bcmode)
        g.set_kick_fusion(fuse)
        g.step(5)
        runs.append(g)
    # the kicked high faces of a cell are recomputed with their owner's
    # arithmetic; only the pairing into fused multiply-adds may differ
    tol = 1e-6 if prec == "fp32" else 1e-14
    for lev in range(nl):
        for name in FIELD_NAMES:
            a, b = runs[0].field(lev, name), runs[1].field(lev, name)
            assert np.max(np.abs(a - b)) <= tol * SCALE[name], (lev, name, float(np.max(np.abs(a - b))))
    fa, fb = runs[0].force(), runs[1].force()
    assert np.max(np.abs(fa[:3] - fb[:3])) <= 1e2 * tol * np.linalg.norm(fa[:3]), (fa, fb)
    assert fa[3] == fb[3]


# The z pass fused with the rebuild, the kick and the end-of-step partials
# against the separate launches: rows of 32, 64 and 128 cells, 96 (a quarter of
# the lanes past the row end), 200 (too long: both sides run the separate
# launches), z extents of one segment, of several with a ragged last one (40)
# and of 2 cells, y extents of 2 to 40 rows.
FINISH_SHAPES = [(32, 16, 8), (64, 12, 6), (96, 10, 40), (128, 40, 6), (128, 2, 2), (64, 18, 70), (200, 6, 4),
                 (16, 4, 34)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", FINISH_SHAPES)
def test_fused_finish_equals_separate(dfm, n, prec):
    _say(f"[fused finish] n={n} {prec}")
    nx, ny, nz = n
    p = dfm.DF_FP32 if prec == "fp32" else dfm.DF_FP64
    runs = []
    for fuse in (False, True):
        g = dfm.Run(nx, ny, nz, dx0=0.05, seed=43, noise_amp=1e-3, precision=p)
        g.set_perturber(0.01, 0.05, 2e-3, 1.3, 0.1)
        g.set_finish_fusion(fuse)
        g.step(6)
        runs.append(g)
    # the same operations in the same order; only the pairing into fused
    # multiply-adds and the grouping of the force partials may differ
    tol = 1e-6 if prec == "fp32" else 1e-14
    for name in FIELD_NAMES:
        a, b = runs[0].field(0, name), runs[1].field(0, name)
        assert np.max(np.abs(a - b)) <= tol * SCALE[name], (name, float(np.max(np.abs(a - b))))
    fa, fb = runs[0].force(), runs[1].force()
    assert np.max(np.abs(fa[:3] - fb[:3])) <= 1e2 * tol * np.linalg.norm(fa[:3]), (fa, fb)
    assert fa[3] == fb[3]
    la, lb = runs[0].force_log(), runs[1].force_log()
    assert la.shape == lb.shape and np.array_equal(la[:, 3], lb[:, 3])  # the same step lengths
    assert np.max(np.abs(la[:, :3] - lb[:, :3])) <= 1e2 * tol * np.max(np.abs(la[:, :3]))


@pytest.mark.parametrize("n,prec,steps", [((24, 24, 24), "fp32", 10), ((128, 64, 96), "fp64", 6),
                                          ((96, 40, 70), "fp32", 6)])
def test_runs_repeat_bitwise(dfm, n, prec, steps):
    # the same run three times gives bitwise the same fields and force: no
    # kernel depends on the order in which its blocks run
    _say(f"[repeat] n={n} {prec} x {steps}")
    nx, ny, nz = n
    p = dfm.DF_FP32 if prec == "fp32" else dfm.DF_FP64
    out = []
    for _ in range(3):
        g = dfm.Run(nx, ny, nz, dx0=0.05, seed=47, noise_amp=1e-3, precision=p)
        g.set_perturber(0.01, 0.05, 2e-3, 0.3, 0.1)
        g.step(steps)
        out.append(({name: g.field(0, name) for name in FIELD_NAMES}, g.force()))
    for other in out[1:]:
        for name in FIELD_NAMES:
            assert np.array_equal(out[0][0][name], other[0][name]), name
        assert np.array_equal(out[0][1], other[1])


def test_fusion_switches_reject_other_values(dfm):
    # through the C ABI itself (the binding passes booleans)
    from paper_1812_03191_amd import _lib

    g = dfm.Run(16, dx0=0.1)
    lib = _lib._load()
    for fn in (lib.df_set_kick_fusion, lib.df_set_transport_fusion, lib.df_set_finish_fusion,
               lib.df_set_step_graphs):
        assert fn(g._h, 0) == 0 and fn(g._h, 1) == 0
        assert fn(g._h, 2) == -1 and fn(g._h, -1) == -1


# ------------------------------------------------------- full single level

def test_config1_parity_100_steps(dfm):
    cfg, steps = inputs.config1()
    _say(f"[parity] config1 32^3 x {steps}")
    o, g = _pair(dfm, cfg)
    assert math.isclose(g.dt(), o.dt(), rel_tol=1e-14)
    o.step(steps)
    g.step(steps)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 1e-11, errs
    fe, fg, fo = _force_err(o, g)
    assert fe < 1e-9, (fg, fo)
    assert fo[0] < 0.0  # cold drag
    assert math.isclose(g.force()[3], o.time, rel_tol=1e-13)


def test_ragged_luminous_parity(dfm):
    # non-cubic, odd multiples of the block width, heat release on
    cfg = inputs.job(24, 1, 0.8, 0.02, 0.1, 2e-3, seed=9)
    cfg.update(nx=40, ny=24, nz=18)
    _say("[parity] ragged 40x24x18 x 30")
    o, g = _pair(dfm, cfg)
    o.step(30)
    g.step(30)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 1e-11, errs
    fe, fg, fo = _force_err(o, g)
    assert fe < 1e-9, (fg, fo)


def test_adiabatic_supersonic_parity(dfm):
    # chi = 0: the Courant limit sets the step (state dependent)
    cfg = inputs.job(32, 1, 2.0, 0.01, 0.1, 0.0, seed=4)
    cfg["chi"] = 0.0
    _say("[parity] adiabatic mach 2 32^3 x 40")
    o, g = _pair(dfm, cfg)
    o.step(40)
    g.step(40)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 1e-11, errs
    assert math.isclose(g.force()[3], o.time, rel_tol=1e-12)


# ------------------------------------------------------------------ nested

@pytest.mark.parametrize("nl,n,steps", [(2, 16, 6), (3, 16, 4), (2, 24, 5), (4, 32, 3)])
def test_nested_parity(dfm, nl, n, steps):
    cfg = inputs.job(n, nl, 0.3, 1e-3, 0.1, 1e-3, seed=3)
    _say(f"[parity] nested {nl} levels of {n}^3 x {steps}")
    o, g = _pair(dfm, cfg)
    o.step(steps)
    g.step(steps)
    errs = _field_errors(o, g, nl)
    assert max(errs.values()) < 1e-11, {k: v for k, v in errs.items() if v > 1e-13}
    fe, fg, fo = _force_err(o, g)
    assert fe < 1e-9, (fg, fo)


# ------------------------------------------- sub-cycling criterion (App. A)

def _fast_coarse(dfm, nl, steps):
    # adiabatic nested run whose level 0 carries an extra -1 in vx outside the
    # refined box (signal speed 2.5 against 1.5 on the finer levels): the
    # criterion takes one level-1 step per coarse step
    from oracle.oracle import Oracle

    kw = dict(nlevels=nl, dx0=0.16, GM=0.01, eps=0.04, L=0.0, mach=0.5, chi=0.0, noise_amp=1e-3, seed=13)
    o = Oracle(16, 16, 16, subcycle=1, **kw)
    g = dfm.Run(16, 16, 16, nlevels=nl, dx0=0.16, seed=13, noise_amp=1e-3)
    g.set_perturber(0.01, 0.04, 0.0, 0.5, 0.0)
    g.set_subcycling(1)
    vx = o.full_field(0, "vx")
    vx[:, :, :3] -= 1.0
    o.set_full_field(0, "vx", vx)
    g.set_field(0, "vx", vx)
    sched = []
    for _ in range(steps):
        o.step(1)
        g.step(1)
        assert g.schedule() == o.schedule()
        sched.append(o.schedule())
    return o, g, sched


@pytest.mark.parametrize("nl,want", [(2, [1]), (3, [1, 2])])
def test_subcycling_criterion_parity(dfm, nl, want):
    _say(f"[parity] sub-cycling criterion, {nl} levels")
    o, g, sched = _fast_coarse(dfm, nl, 3)
    assert sched[0] == want, sched
    errs = _field_errors(o, g, nl)
    assert max(errs.values()) < 1e-11, {k: v for k, v in errs.items() if v > 1e-13}
    fe, fg, fo = _force_err(o, g)
    assert fe < 1e-9, (fg, fo)
    assert abs(g.force()[3] - o.time) < 1e-14 * o.time


def test_subcycling_criterion_keeps_two_on_nested_setup(dfm):
    # limits halving level by level: the criterion keeps xi = 2 and the run is
    # bitwise the default one
    cfg = inputs.job(16, 3, 0.3, 1e-3, 0.1, 1e-3, seed=3)
    _say("[parity] sub-cycling criterion on the nested setup")
    _, a = _pair(dfm, cfg)
    _, b = _pair(dfm, cfg)
    a.set_subcycling(1)
    for _ in range(3):
        a.step(1)
        b.step(1)
        assert a.schedule() == [2, 2]
    for lev in range(3):
        for name in FIELD_NAMES:
            assert np.array_equal(a.field(lev, name), b.field(lev, name)), (lev, name)
    assert np.array_equal(a.force(), b.force())


# ------------------------------------- the paper's boundary list (Sect. 3.4)

def _wall_pair(dfm, n, seed, **kw):
    # random state of _random_pair with the wall faces at zero normal velocity
    from oracle.oracle import Oracle

    o0, g = _random_pair(dfm, n, seed, **kw)
    nx, ny, nz = n
    o = Oracle(nx, ny, nz, dx0=0.05, GM=kw.get("GM", 0.01), eps=kw.get("eps", 0.05), L=kw.get("L", 2e-3),
               mach=kw.get("mach", 0.5), chi=kw.get("chi", 0.1), noise_amp=0.0, bcmode=1)
    g.set_boundaries(1)
    for name in FIELD_NAMES:
        a = g.field(0, name)
        if name == "vy":
            a[:, 0, :] = 0.0
            a[:, -1, :] = 0.0
        if name == "vz":
            a[0, :, :] = 0.0
            a[-1, :, :] = 0.0
        g.set_field(0, name, a)
        o.set_full_field(0, name, a)
    return o, g


@pytest.mark.parametrize("stage,dt", STAGE_CASES)
@pytest.mark.parametrize("n", [(16, 16, 16), (20, 12, 18)])
def test_wall_boundaries_stage_parity(dfm, stage, dt, n):
    _say(f"[wall parity] {stage} n={n}")
    o, g = _wall_pair(dfm, n, seed=31)
    o.stage(stage, dt)
    g.stage(stage, dt)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 1e-13, {k: v for k, v in errs.items() if v > 1e-14}


@pytest.mark.parametrize("nl,n,steps", [(1, 32, 60), (2, 16, 6), (3, 16, 4)])
def test_wall_boundaries_parity(dfm, nl, n, steps):
    # whole steps under the boundary list of Sect. 3.4, gamma 1.4 and eps 0 as in
    # the paper; on 16^3 the finer levels' ghost shells reach past level 0, so
    # their fill reads level 0's mirror images
    from oracle.oracle import Oracle

    cfg = dict(inputs.job(n, nl, 0.4, 5e-3, 0.1, 1e-3, seed=17, gamma=1.4), eps=0.0)
    _say(f"[wall parity] {nl} levels of {n}^3 x {steps}")
    c = cfg
    o = Oracle(n, n, n, nlevels=nl, dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"], seed=c["seed"],
               noise_amp=c["noise_amp"], GM=c["GM"], eps=0.0, L=c["L"], mach=c["mach"], chi=c["chi"], bcmode=1)
    g = dfm.Run(n, n, n, nlevels=nl, dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"], seed=c["seed"],
                noise_amp=c["noise_amp"])
    g.set_boundaries(1)
    g.set_perturber(c["GM"], 0.0, c["L"], c["mach"], c["chi"])
    o.step(steps)
    g.step(steps)
    errs = _field_errors(o, g, nl)
    assert max(errs.values()) < 1e-11, {k: v for k, v in errs.items() if v > 1e-13}
    fe, fg, fo = _force_err(o, g)
    assert fe < 1e-9, (fg, fo)


# ------------------------------------------- artificial viscosity (SubStep2)

@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("n", [(16, 16, 16), (20, 12, 18)])
def test_viscosity_stage_parity(dfm, n, walls):
    from oracle.oracle import Oracle

    _say(f"[viscosity parity] stage n={n} walls={walls}")
    if walls:
        o0, g = _wall_pair(dfm, n, seed=37)
    else:
        o0, g = _random_pair(dfm, n, seed=37)
    nx, ny, nz = n
    o = Oracle(nx, ny, nz, dx0=0.05, GM=0.01, eps=0.05, L=2e-3, mach=0.5, chi=0.1, noise_amp=0.0,
               bcmode=1 if walls else 0, visc=2.0)
    for name in FIELD_NAMES:
        o.set_full_field(0, name, g.field(0, name))
    g.set_viscosity(2.0)
    # velocity departures of 1e-3 over 0.05 cells: dt large enough for q to show
    o.stage("viscosity", 0.5)
    g.stage("viscosity", 0.5)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 1e-13, {k: v for k, v in errs.items() if v > 1e-14}
    ref = o0.full_field(0, "e")
    assert np.max(np.abs(o.full_field(0, "e") - ref)) > 1e-9  # the stage did act


@pytest.mark.parametrize("nl,n,steps,walls", [(1, 32, 40, False), (2, 16, 6, False), (1, 24, 20, True)])
def test_viscosity_run_parity(dfm, nl, n, steps, walls):
    # supersonic (Mach 2) runs with the viscosity on, whole steps
    from oracle.oracle import Oracle

    c = inputs.job(n, nl, 2.0, 0.01, 0.1, 1e-3, seed=19)
    _say(f"[viscosity parity] {nl} levels of {n}^3 x {steps} walls={walls}")
    o = Oracle(n, n, n, nlevels=nl, dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"], seed=c["seed"],
               noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"], L=c["L"], mach=c["mach"], chi=c["chi"],
               bcmode=1 if walls else 0, visc=2.0)
    g = dfm.Run(n, n, n, nlevels=nl, dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"], seed=c["seed"],
                noise_amp=c["noise_amp"])
    g.set_viscosity(2.0)
    if walls:
        g.set_boundaries(1)
    g.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
    o.step(steps)
    g.step(steps)
    errs = _field_errors(o, g, nl)
    assert max(errs.values()) < 1e-11, {k: v for k, v in errs.items() if v > 1e-13}
    fe, fg, fo = _force_err(o, g)
    assert fe < 1e-9, (fg, fo)


@pytest.mark.parametrize("gf", [11, 12])
def test_nested_wider_ghosts_parity(dfm, gf):
    # an odd width leaves one child of the outermost coarse hosts outside the
    # stored fine box
    cfg = inputs.job(16, 2, 0.6, 5e-3, 0.1, 1e-3, seed=8)
    _say(f"[parity] nested ghost width {gf}")
    o, g = _pair(dfm, cfg, gf=gf)
    o.step(4)
    g.step(4)
    errs = _field_errors(o, g, 2)
    assert max(errs.values()) < 1e-11, errs


def test_uniform_flow_exact_on_gpu(dfm):
    g = dfm.Run(16, nlevels=3, dx0=0.2, noise_amp=0.0)
    g.set_perturber(0.0, 0.0, 0.0, 1.3, 0.1)
    g.step(5)
    for lev in range(3):
        assert np.all(g.field(lev, "rho") == 1.0)
        assert np.all(g.field(lev, "e") == E0)
        assert np.all(g.field(lev, "vx") == -1.3)
        assert np.all(g.field(lev, "vy") == 0.0)
    assert np.all(g.force()[:3] == 0.0)


def test_health_flag_reports_negative_density(dfm):
    g = dfm.Run(16, dx0=0.05, noise_amp=0.0)
    g.set_perturber(0.01, 0.1, 0.0, 0.5, 0.1)
    rho = g.field(0, "rho")
    rho[3, 4, 5] = -1.0
    g.set_field(0, "rho", rho)
    g.step(1)
    with pytest.raises(dfm.DFError) as ei:
        g.force()
    assert ei.value.code == -5


# ------------------------------------------------------------ full sizes

def test_config2_full_size_parity_short(dfm):
    # 128^3 at the benchmark's launch configuration: all fields after 4 steps
    cfg, _ = inputs.config2()
    _say("[parity] config2 128^3 x 4")
    o, g = _pair(dfm, cfg)
    o.step(4)
    g.step(4)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 1e-12, errs
    fe, fg, fo = _force_err(o, g)
    assert fe < 1e-10, (fg, fo)


def test_config2_full_run_properties(dfm):
    # 500 steps at 128^3: y/z mirror symmetry of the solution, positivity,
    # drag of the cold run and thrust of the heating force (eq. 5)
    cfg, steps = inputs.config2()
    _say("[properties] config2 128^3 x 500 (hot and cold)")
    runs = {}
    for L in (0.0, cfg["L"]):
        g = dfm.Run(128, dx0=cfg["dx0"], seed=cfg["seed"], noise_amp=0.0)
        g.set_perturber(cfg["GM"], cfg["eps"], L, cfg["mach"], cfg["chi"])
        g.step(steps)
        runs[L] = g
    cold, hot = runs[0.0].force(), runs[cfg["L"]].force()
    assert cold[0] < 0.0
    assert hot[0] - cold[0] > 0.0
    rho = runs[cfg["L"]].field(0, "rho")
    assert np.all(rho > 0)
    assert np.max(np.abs(rho - rho[:, ::-1, :])) < 1e-13
    assert np.max(np.abs(rho - rho[::-1, :, :])) < 1e-13
    assert abs(hot[1]) < 1e-9 * abs(hot[0]) and abs(hot[2]) < 1e-9 * abs(hot[0])


# ---------------------------------------------------- FP32 departure storage

def _pair32(dfm, cfg):
    from oracle.oracle import Oracle

    c = dict(cfg)
    o = Oracle(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"],
               cfl=c["cfl"], seed=c["seed"], noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"],
               L=c["L"], mach=c["mach"], chi=c["chi"])
    g = dfm.Run(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"],
                cfl=c["cfl"], seed=c["seed"], noise_amp=c["noise_amp"], precision=dfm.DF_FP32)
    g.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
    return o, g


@pytest.mark.parametrize("stage,dt", STAGE_CASES)
def test_stage_parity_fp32(dfm, stage, dt):
    # departures of ~1e-3 stored in FP32: ~1e-10 absolute per stage
    from oracle.oracle import Oracle

    n = (20, 12, 18)
    _say(f"[stage parity fp32] {stage}")
    o, g64 = _random_pair(dfm, n, seed=23)
    g = dfm.Run(*n, dx0=0.05, noise_amp=0.0, precision=dfm.DF_FP32)
    g.set_perturber(0.01, 0.05, 2e-3, 0.5, 0.1)
    for name in FIELD_NAMES:
        g.set_field(0, name, g64.field(0, name))
    o.stage(stage, dt)
    g.stage(stage, dt)
    errs = _field_errors(o, g, 1)
    assert max(errs.values()) < 2e-8, errs


def _fp32_report(o, g, nlevels):
    fo, fg = o.force(), g.force()[:3]
    to, tg = o.totals()[:3], g.totals()
    rep = {"force_rel": float(abs(fg[0] - fo[0]) / abs(fo[0])),
           "mass_rel": float(abs(tg[0] - to[0]) / to[0]),
           "eint_rel": float(abs(tg[1] - to[1]) / to[1]),
           "ekin_rel": float(abs(tg[2] - to[2]) / max(to[2], 1e-300))}
    drho = max(float(np.max(np.abs(g.field(l, "rho") - o.field(l, "rho")))) for l in range(nlevels))
    rep["rho_abs"] = drho
    return rep


def test_fp32_config1_force_error(dfm):
    # FP32 departures vs the FP64 oracle after 100 steps: force within 1e-4
    cfg, steps = inputs.config1()
    _say("[fp32] config1 32^3 x 100")
    o, g = _pair32(dfm, cfg)
    o.step(steps)
    g.step(steps)
    rep = _fp32_report(o, g, 1)
    _say(f"[fp32] config1 errors {rep}")
    assert rep["force_rel"] < 1e-4, rep
    assert rep["mass_rel"] < 1e-7, rep
    assert rep["eint_rel"] < 1e-6 and rep["ekin_rel"] < 1e-6, rep


def test_fp32_nested_force_error(dfm):
    cfg = inputs.job(32, 3, 0.3, 1e-3, 0.1, 1e-3, seed=3)
    _say("[fp32] nested 3 x 32^3 x 20")
    o, g = _pair32(dfm, cfg)
    o.step(20)
    g.step(20)
    rep = _fp32_report(o, g, 3)
    _say(f"[fp32] nested errors {rep}")
    assert rep["force_rel"] < 1e-4, rep
    assert rep["mass_rel"] < 1e-6 and rep["eint_rel"] < 1e-6 and rep["ekin_rel"] < 1e-6, rep
