"""The paper's quadrant (Sect. 3.4) on the HIP path: the domain y > 0, z > 0
bounded by the perturber's mirror planes, every nested level anchored at
them, finer levels' entries beyond the planes kept as mirror images.
Parity with the FP64 oracle's quadrant (every field of every level within
1e-11 of its scale, the force of the whole gas within 1e-9) on one level, on
the central-half hierarchy and on the quarter hierarchy of Sects. 4.1.3 and
4.2.2; a quadrant run against the quarter y, z > 0 of the full box on the
GPU; FP32 storage against the oracle; an engine job of this shape bitwise
equal to the job run alone."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NAMES = ("rho", "e", "vx", "vy", "vz")


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


BASE = dict(gamma=1.4, GM=5e-3, eps=0.0, L=2e-3, mach=0.4, chi=0.1)


def _gpu(dfm, n, nl, n1, dx0, *, quadrant, noise, precision=0, seed=3):
    shape = (n, n // 2, n // 2) if quadrant else (n, n, n)
    m1 = None
    if n1:
        m1 = (n1, n1 // 2, n1 // 2) if quadrant else (n1, n1, n1)
    g = dfm.Run(*shape, nlevels=nl, dx0=dx0, gamma=BASE["gamma"], seed=seed, noise_amp=noise,
                precision=precision, n1=m1, quadrant=quadrant)
    g.set_boundaries(1)
    g.set_perturber(BASE["GM"], BASE["eps"], BASE["L"], BASE["mach"], BASE["chi"])
    return g


def _oracle(n, nl, n1, dx0, noise, seed=3):
    from oracle.oracle import Oracle

    return Oracle(n, n // 2, n // 2, nlevels=nl, dx0=dx0, seed=seed, noise_amp=noise, bcmode=1,
                  n1=(n1, n1 // 2, n1 // 2) if n1 else None, quadrant=True, **BASE)


CASES = [  # (ground cells along x, levels, finer-level cells along x, steps, dx0)
    (32, 1, None, 12, 0.05),
    (32, 2, None, 4, 0.16),
    (64, 3, 32, 3, 0.16),
    (32, 4, None, 2, 0.32),
]


@pytest.mark.parametrize("n,nl,n1,steps,dx0", CASES)
def test_quadrant_parity_with_oracle(dfm, n, nl, n1, steps, dx0):
    _say(f"[quadrant] {n}x{n // 2}x{n // 2}, {nl} levels, n1 {n1}, {steps} steps vs oracle")
    g = _gpu(dfm, n, nl, n1, dx0, quadrant=True, noise=1e-4)
    o = _oracle(n, nl, n1, dx0, 1e-4)
    g.step(steps)
    o.step(steps)
    e0 = 1.0 / (BASE["gamma"] * (BASE["gamma"] - 1.0))
    errs = {}
    for lev in range(nl):
        for name in NAMES:
            a, b = g.field(lev, name), o.full_field(lev, name)
            assert a.shape == b.shape, (lev, name, a.shape, b.shape)
            errs[(lev, name)] = float(np.max(np.abs(a - b))) / (e0 if name == "e" else 1.0)
    assert max(errs.values()) < 1e-11, {k: v for k, v in errs.items() if v > 1e-13}
    fg, fo = g.force()[:3], o.force()
    assert fg[1] == 0.0 and fg[2] == 0.0
    assert abs(fg[0] - fo[0]) <= 1e-9 * abs(fo[0]), (fg, fo)
    assert abs(g.force()[3] - o.time) <= 1e-12 * o.time
    tg, to = g.totals(), o.totals()[:3]
    assert np.max(np.abs(tg[:3] - to) / np.abs(to)) < 1e-12, (tg, to)


def test_quadrant_parity_on_the_papers_level_shapes(dfm):
    # the level shapes of Sect. 4.2.2 as the quadrant: ground 64 x 64 x 128 (128
    # along the flow, here x), finer levels 32 x 32 x 64 (3 levels)
    _say("[quadrant] 128x64x64 + 2 levels of 64x32x32 vs oracle, 2 steps")
    g = _gpu(dfm, 128, 3, 64, 0.16, quadrant=True, noise=1e-4)
    o = _oracle(128, 3, 64, 0.16, 1e-4)
    g.step(2)
    o.step(2)
    e0 = 1.0 / (BASE["gamma"] * (BASE["gamma"] - 1.0))
    for lev in range(3):
        for name in NAMES:
            a, b = g.field(lev, name), o.full_field(lev, name)
            assert a.shape == b.shape, (lev, name)
            assert float(np.max(np.abs(a - b))) / (e0 if name == "e" else 1.0) < 1e-11, (lev, name)
    fg, fo = g.force()[0], o.force()[0]
    assert abs(fg - fo) <= 1e-9 * abs(fo), (fg, fo)


@pytest.mark.parametrize("n,nl,n1,steps,dx0", [(32, 2, None, 4, 0.16), (64, 3, 32, 3, 0.16)])
def test_quadrant_is_a_quarter_of_the_full_box(dfm, n, nl, n1, steps, dx0):
    # no noise: the full box then holds the quadrant's mirror images
    _say(f"[quadrant] {n}^3 full box vs quadrant, {nl} levels, n1 {n1}")
    full = _gpu(dfm, n, nl, n1, dx0, quadrant=False, noise=0.0)
    quad = _gpu(dfm, n, nl, n1, dx0, quadrant=True, noise=0.0)
    full.step(steps)
    quad.step(steps)
    for lev in range(nl):
        h = (n if lev == 0 or not n1 else n1) // 2
        for name in NAMES:
            a = full.field(lev, name)[h:, h:, :]
            b = quad.field(lev, name)
            assert a.shape == b.shape, (lev, name)
            assert float(np.max(np.abs(a - b))) < 1e-13, (lev, name)
    ff, fq = full.force(), quad.force()
    assert abs(fq[0] - ff[0]) <= 1e-11 * abs(ff[0]), (fq, ff)


def test_quadrant_fp32_against_oracle(dfm):
    _say("[quadrant] FP32, 64x32x32 + 2 levels of 32x16x16, 6 steps")
    g = _gpu(dfm, 64, 3, 32, 0.16, quadrant=True, noise=1e-4, precision=1)
    o = _oracle(64, 3, 32, 0.16, 1e-4)
    g.step(6)
    o.step(6)
    fg, fo = g.force()[0], o.force()[0]
    rel = abs(fg - fo) / abs(fo)
    _say(f"[quadrant] FP32 force error {rel:.2e}")
    assert rel < 1e-4


def test_quadrant_engine_job_equals_run(dfm):
    import torch

    cfg = dict(nx=32, ny=16, nz=16, nlevels=2, dx0=0.16, gamma=BASE["gamma"], cfl=0.4, seed=4,
               noise_amp=1e-4, quadrant=True, **{k: BASE[k] for k in ("GM", "eps", "L", "mach", "chi")})
    eng = dfm.Engine(1 << 30)
    s = eng.admit(cfg, 4, precision=1)
    eng.step(2)
    torch.cuda.synchronize()
    assert s in eng.poll()
    r = dfm.Run(32, 16, 16, nlevels=2, dx0=0.16, gamma=BASE["gamma"], seed=4, noise_amp=1e-4, precision=1,
                quadrant=True)
    r.set_perturber(BASE["GM"], BASE["eps"], BASE["L"], BASE["mach"], BASE["chi"])
    r.step(4)
    for lev in range(2):
        for name in NAMES:
            assert np.array_equal(eng.field(s, lev, name, r.shape(name, lev)), r.field(lev, name)), (lev, name)
    assert np.array_equal(eng.force(s), r.force())
