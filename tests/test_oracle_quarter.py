"""Pins of the oracle on the mesh hierarchy of Sects. 4.1.3 and 4.2.2, whose
first refined level covers a quarter of the ground level along each
dimension (the finer levels have half the ground level's cells, level l+1
covering the central n_{l+1}/2 cells of level l).  The same invariants as on
the central-half hierarchy: uniform flow exactly, composite mass to
round-off, restriction of a prolongation, linear data, mirror symmetry, ghost
width, and Newton's shell theorem across the quarter's frontier.  CPU only."""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle

GAMMA = 5.0 / 3.0
E0 = 1.0 / (GAMMA * (GAMMA - 1.0))


def test_rejects_finer_levels_that_do_not_fit():
    with pytest.raises(ValueError):
        Oracle(32, 32, 32, nlevels=2, dx0=0.1, n1=(18, 16, 16))  # not a multiple of 4
    with pytest.raises(ValueError):
        Oracle(16, 16, 16, nlevels=2, dx0=0.1, n1=(40, 16, 16))  # wider than level 0


def test_uniform_flow_stays_uniform():
    o = Oracle(32, 32, 32, nlevels=3, dx0=0.2, GM=0.0, L=0.0, noise_amp=0.0, mach=1.3, chi=0.1,
               n1=(16, 16, 16))
    o.step(5)
    for lev in range(3):
        s = o.state(lev, ghosts=True)
        assert s["rho"].shape == ((38, 38, 38) if lev == 0 else (36, 36, 36))
        assert np.all(s["rho"] == 1.0), lev
        assert np.all(s["e"] == E0), lev
        assert np.all(s["vx"] == -1.3), lev
        assert np.all(s["vy"] == 0.0) and np.all(s["vz"] == 0.0), lev
    assert np.all(o.force() == 0.0)


@pytest.mark.parametrize("nlevels", [2, 3])
def test_composite_mass_conservation(nlevels):
    o = Oracle(32, 32, 32, nlevels=nlevels, dx0=0.16, GM=0.02, eps=0.04, L=2e-3, mach=0.9, chi=0.1,
               noise_amp=1e-3, seed=11, n1=(16, 16, 16))
    m0 = o.totals()[0]
    o.step(4)
    m1, _, _, inflow = o.totals()
    assert abs((m1 - m0) - inflow) < 1e-14 * m0 * 16, (m1 - m0, inflow)


def test_covered_cells_hold_restricted_fine_data():
    # level 1 (16^3) covers coarse cells 12..19 of the 32^3 ground level
    o = Oracle(32, 32, 32, nlevels=2, dx0=0.16, GM=0.02, eps=0.04, L=2e-3, mach=0.9, chi=0.1,
               noise_amp=1e-3, seed=11, n1=(16, 16, 16))
    o.step(1)
    rho_c = o.field(0, "rho")
    fine = o.field(1, "rho")
    restricted = fine.reshape(8, 2, 8, 2, 8, 2).mean(axis=(1, 3, 5))
    assert np.max(np.abs(rho_c[12:20, 12:20, 12:20] - restricted)) < 1e-15


def test_restriction_of_prolongation_is_identity():
    o = Oracle(32, 32, 32, nlevels=2, dx0=0.1, GM=0.0, noise_amp=0.0, n1=(16, 16, 16))
    rng = np.random.default_rng(3)
    sh = (32 + 6, 32 + 6, 32 + 6)
    coarse = {}
    for name in ("rho", "e", "vx", "vy", "vz"):
        a = 1.0 + 0.1 * rng.standard_normal(sh)
        coarse[name] = a
        o.set_field(0, name, a, ghosts=True)
    o.prolong_all(0)
    o.commmean(0)
    sl = slice(3 + 12, 3 + 20)
    for name in ("rho", "e", "vx", "vy", "vz"):
        got = o.field(0, name, ghosts=True)
        d = np.max(np.abs(got[sl, sl, sl] - coarse[name][sl, sl, sl]))
        assert d < 1e-15 * 4, (name, d)


def test_prolongation_reproduces_linear_data():
    # fine positions of the quarter level: centred on the same vertex, half the
    # cell size, n1 cells
    n, n1, dx = 32, 16, 0.1
    o = Oracle(n, n, n, nlevels=2, dx0=dx, GM=0.0, noise_amp=0.0, n1=(n1, n1, n1))
    g = 3
    idx = np.arange(-g, n + g)
    xc = (idx - n / 2 + 0.5) * dx
    xf = (idx - n / 2) * dx
    a, b, c = 0.3, -0.2, 0.7

    def lin(x, y, z):
        return 1.0 + a * x[None, None, :] + b * y[None, :, None] + c * z[:, None, None]

    o.set_field(0, "rho", lin(xc, xc, xc), ghosts=True)
    o.set_field(0, "vy", lin(xc, xf, xc), ghosts=True)
    o.prolong_all(0)
    gf = 10
    fidx = np.arange(-gf, n1 + gf)
    fdx = dx / 2
    fxc = (fidx - n1 / 2 + 0.5) * fdx
    fxf = (fidx - n1 / 2) * fdx
    for name, want in (("rho", lin(fxc, fxc, fxc)), ("vy", lin(fxc, fxf, fxc))):
        got = o.field(1, name, ghosts=True)
        assert np.max(np.abs(got - want)) < 1e-14, name


def test_mirror_symmetry_and_ghost_width():
    kw = dict(nlevels=3, dx0=0.16, GM=0.01, eps=0.02, L=2e-3, noise_amp=0.0, mach=0.8, chi=0.1,
              n1=(16, 16, 16))
    runs = {gf: Oracle(32, 32, 32, gf=gf, **kw) for gf in (10, 12)}
    for r in runs.values():
        r.step(3)
    o = runs[10]
    for lev in range(3):
        for name in ("rho", "e", "vx"):
            a = o.field(lev, name)
            assert np.array_equal(a, a[:, ::-1, :]), (lev, name)
            assert np.array_equal(a, a[::-1, :, :]), (lev, name)
            assert np.array_equal(a, runs[12].field(lev, name)), (lev, name)
    F = o.force()
    assert F[0] != 0.0 and abs(F[1]) <= 1e-12 * abs(F[0]) and abs(F[2]) <= 1e-12 * abs(F[0])


def _blob_error(n, n1, dx0):
    # the blob sits on the x_max face of level 1, which covers the central
    # quarter [-n dx0 / 8, n dx0 / 8] of level 0
    C, s, amp = (n * dx0 / 8.0, 0.05, -0.03), 0.12, 1e-2
    o = Oracle(n, n, n, nlevels=2, dx0=dx0, GM=0.01, eps=0.0, noise_amp=0.0, n1=(n1, n1, n1))
    for lev, (m, dx) in enumerate(((n, dx0), (n1, dx0 / 2))):
        x = (np.arange(m) - m / 2 + 0.5) * dx
        X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
        o.set_field(lev, "rho", 1.0 + amp * np.exp(-((X - C[0]) ** 2 + (Y - C[1]) ** 2 + (Z - C[2]) ** 2) / (2 * s * s)))
    F = o.force()
    mass = amp * (2.0 * math.pi) ** 1.5 * s ** 3
    Cv = np.asarray(C)
    Fs = 0.01 * mass * Cv / np.linalg.norm(Cv) ** 3
    return float(np.max(np.abs(F - Fs)) / np.linalg.norm(Fs))


def test_force_across_quarter_frontier_converges_to_point_mass():
    e1 = _blob_error(96, 48, 0.08)
    e2 = _blob_error(192, 96, 0.04)
    assert e1 < 5e-3 and e2 < e1 / 3.0, (e1, e2)
