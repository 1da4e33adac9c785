"""The hierarchy of the paper's Sects. 4.1.3 and 4.2.2 on the HIP path: finer
levels with half the ground level's cells, the first covering the central
quarter of the ground level.  Parity with the FP64 oracle (every field of
every level within 1e-11 of its scale, the force within 1e-9; FP32 storage:
force within 1e-4), in the default boundaries and in the paper's own setup
(gamma 1.4, eps 0, the boundary list of Sect. 3.4), and an engine job of this
shape bitwise equal to the job run alone."""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu

FIELD_NAMES = ("rho", "e", "vx", "vy", "vz")


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


def _pair(dfm, c, *, bcmode=0, precision=0):
    from oracle.oracle import Oracle

    o = Oracle(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"],
               seed=c["seed"], noise_amp=c["noise_amp"], GM=c["GM"], eps=c["eps"], L=c["L"], mach=c["mach"],
               chi=c["chi"], bcmode=bcmode, n1=c["n1"])
    g = dfm.Run(c["nx"], c["ny"], c["nz"], nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"], cfl=c["cfl"],
                seed=c["seed"], noise_amp=c["noise_amp"], precision=precision, n1=c["n1"])
    if bcmode:
        g.set_boundaries(1)
    g.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
    return o, g


def _errors(o, g, nl, gamma):
    e0 = 1.0 / (gamma * (gamma - 1.0))
    scale = {"rho": 1.0, "e": e0, "vx": 1.0, "vy": 1.0, "vz": 1.0}
    errs = {}
    for lev in range(nl):
        for name in FIELD_NAMES:
            a, b = g.field(lev, name), o.full_field(lev, name)
            assert a.shape == b.shape, (lev, name, a.shape, b.shape)
            errs[(lev, name)] = float(np.max(np.abs(a - b))) / scale[name]
    return errs


CASES = [  # (ground cells, levels, Mach, boundary mode, coarse steps)
    (32, 3, 0.4, 0, 6),
    (64, 4, 0.3, 0, 3),
    (32, 3, 0.2, 1, 6),
]


@pytest.mark.parametrize("n0,nl,mach,bcmode,steps", CASES)
def test_quarter_hierarchy_parity(dfm, n0, nl, mach, bcmode, steps):
    _say(f"[quarter] ground {n0}^3 + {nl - 1} levels of {n0 // 2}^3, Mach {mach}, bc {bcmode}, {steps} steps")
    if bcmode:
        c = inputs.paper_mesh(n0, nl, mach, 0.1, GM=5e-3, L=1e-3, seed=21, noise_amp=1e-4)
    else:
        c = inputs.job(n0, nl, mach, 5e-3, 0.1, 1e-3, seed=21, n1=n0 // 2)
    o, g = _pair(dfm, c, bcmode=bcmode)
    o.step(steps)
    g.step(steps)
    errs = _errors(o, g, nl, c["gamma"])
    assert max(errs.values()) < 1e-11, {k: v for k, v in errs.items() if v > 1e-13}
    fg, fo = g.force()[:3], o.force()
    assert np.max(np.abs(fg - fo)) <= 1e-9 * np.linalg.norm(fo), (fg, fo)
    assert abs(g.force()[3] - o.time) <= 1e-12 * o.time


def test_quarter_hierarchy_fp32_against_oracle(dfm):
    c = inputs.paper_mesh(64, 4, 0.2, 0.1, GM=2e-3, seed=22, noise_amp=1e-4)
    _say("[quarter] FP32, ground 64^3 + 3 levels of 32^3, paper setup, 10 steps")
    o, g = _pair(dfm, c, bcmode=1, precision=1)
    o.step(10)
    g.step(10)
    fg, fo = g.force()[:3], o.force()
    rel = float(abs(fg[0] - fo[0]) / abs(fo[0]))
    tg, to = g.totals(), o.totals()[:3]
    _say(f"[quarter] FP32 force error {rel:.2e}, mass error {abs(tg[0] - to[0]) / to[0]:.2e}")
    assert rel < 1e-4
    assert abs(tg[0] - to[0]) < 1e-6 * to[0]


def test_quarter_hierarchy_engine_job_equals_run(dfm):
    c = inputs.job(32, 3, 0.5, 2e-3, 0.1, 1e-3, seed=23, n1=16)
    eng = dfm.Engine(1 << 30)
    s = eng.admit(c, 4, precision=1)
    eng.step(2)
    import torch

    torch.cuda.synchronize()
    assert s in eng.poll()
    r = dfm.Run(32, nlevels=3, dx0=c["dx0"], seed=c["seed"], noise_amp=c["noise_amp"], precision=1, n1=c["n1"])
    r.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
    r.step(4)
    for lev in range(3):
        for name in FIELD_NAMES:
            shp = r.shape(name, lev)
            assert np.array_equal(eng.field(s, lev, name, shp), r.field(lev, name)), (lev, name)
    assert np.array_equal(eng.force(s), r.force())
