"""Pins of the oracle's force sum (eq. 18) and of the transport stage's
conservation, against values the mathematics fixes without evaluating the
oracle's own formulas.  CPU only.

* Newton's shell theorem: a spherically symmetric over-density pulls a point
  outside it as its whole mass placed at its centre.  A Gaussian blob sampled
  at the cell centres is integrated by the midpoint rule to within
  exp(-2 pi^2 s^2 / dx^2) (spectral accuracy of a smooth integrand), so on one
  level eq. 18 must give G M m C / |C|^3 to round-off.  This fixes the cell
  volume, the exponent 3/2 of the softened distance (eps = 0 here), the sign
  and the cell-centre positions.
* The same blob straddling the frontier of a finer level: the composite sum
  (finer cells where they exist, uncovered coarse cells elsewhere) converges to
  the same value at second order in the cell size, which fixes which coarse
  cells count as covered.
* One cell: a single departure d rho at a known cell is the softened point
  mass G M d rho dx^3 r / (r^2 + eps^2)^(3/2) (eq. 16 differentiated), and the
  same departure in a covered coarse cell pulls nothing.
* Transport (Sect. 3.2.3): the flux form moves energy and the cell momenta
  between cells only, so with a departure confined to the interior their sums
  are unchanged to round-off by the transport stage, the momentum read back
  through the rebuilt face velocities.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle

GM = 0.01


def _centres(n, dx):
    return (np.arange(n) - n / 2 + 0.5) * dx


def _blob(n, dx, C, s, amp):
    x = _centres(n, dx)
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    r2 = (X - C[0]) ** 2 + (Y - C[1]) ** 2 + (Z - C[2]) ** 2
    return 1.0 + amp * np.exp(-r2 / (2.0 * s * s))


def _shell_value(C, s, amp):
    m = amp * (2.0 * math.pi) ** 1.5 * s ** 3
    C = np.asarray(C, dtype=float)
    return GM * m * C / np.linalg.norm(C) ** 3


def test_force_of_gaussian_blob_is_point_mass_single_level():
    n, dx = 48, 0.05
    C, s, amp = (0.45, -0.35, 0.3), 0.075, 1e-2  # |C| = 8.5 s; 10 s from the box edge
    o = Oracle(n, n, n, dx0=dx, GM=GM, eps=0.0, noise_amp=0.0)
    o.set_field(0, "rho", _blob(n, dx, C, s, amp))
    F = o.force()
    Fs = _shell_value(C, s, amp)
    assert np.max(np.abs(F - Fs)) <= 1e-9 * np.linalg.norm(Fs), (F, Fs)


def _two_level_blob_error(n, dx0):
    # level 1 covers [-n dx0 / 4, n dx0 / 4]^3; the blob is centred on its
    # x_max frontier plane, so half of its mass lies on each level
    C, s, amp = (0.96, 0.1, -0.05), 0.12, 1e-2
    o = Oracle(n, n, n, nlevels=2, dx0=dx0, GM=GM, eps=0.0, noise_amp=0.0)
    assert math.isclose(n * dx0 / 4.0, C[0])
    for lev in range(2):
        o.set_field(lev, "rho", _blob(n, dx0 / 2 ** lev, C, s, amp))
    F = o.force()
    Fs = _shell_value(C, s, amp)
    return float(np.max(np.abs(F - Fs)) / np.linalg.norm(Fs)), F, Fs


def test_force_of_blob_across_frontier_converges_to_point_mass():
    e1, F1, Fs = _two_level_blob_error(48, 0.08)
    e2, F2, _ = _two_level_blob_error(96, 0.04)
    # counting the covered coarse cells as well (or dropping the finer level)
    # would be off by about half the blob's pull
    assert e1 < 5e-3, (e1, F1, Fs)
    assert e2 < e1 / 3.0, (e1, e2)


@pytest.mark.parametrize("eps", [0.0, 0.03])
def test_force_of_one_cell_is_softened_point_mass(eps):
    n, dx0, d = 16, 0.1, 0.25
    o = Oracle(n, n, n, nlevels=2, dx0=dx0, GM=GM, eps=eps, noise_amp=0.0)
    # an uncovered level-0 cell (i, j, k) and a covered one
    i, j, k = 13, 5, 9
    x = _centres(n, dx0)
    rho = np.ones((n, n, n))
    rho[k, j, i] += d
    o.set_field(0, "rho", rho)
    r = np.array([x[i], x[j], x[k]])
    want = GM * d * dx0 ** 3 * r / (r @ r + eps * eps) ** 1.5
    F = o.force()
    assert np.max(np.abs(F - want)) <= 1e-14 * np.linalg.norm(want), (F, want)
    rho = np.ones((n, n, n))
    rho[7, 9, 5] += d  # inside [n/4, 3n/4): covered by level 1
    o.set_field(0, "rho", rho)
    assert np.all(o.force() == 0.0)


def _bump(n, lo, hi):
    # smooth bump with support exactly inside cells [lo, hi) of a row
    t = np.zeros(n)
    i = np.arange(lo, hi)
    t[lo:hi] = np.sin(math.pi * (i - lo + 0.5) / (hi - lo)) ** 2
    return t


def _face_sum(v, rho, axis):
    """sum over faces of v_f (rho_below + rho_above), interior faces with both
    cells and the two boundary faces with their one cell"""
    n = rho.shape[axis]
    lo = np.take(v, 0, axis=axis) * np.take(rho, 0, axis=axis)
    hi = np.take(v, n, axis=axis) * np.take(rho, n - 1, axis=axis)
    inner = np.take(v, np.arange(1, n), axis=axis) * (
        np.take(rho, np.arange(0, n - 1), axis=axis) + np.take(rho, np.arange(1, n), axis=axis))
    return float(np.sum(inner) + np.sum(lo) + np.sum(hi))


def _cell_momentum(v, rho, axis):
    """sum over cells of rho_c (v_low face + v_high face): the sum of the two
    cell momenta the transport moves"""
    n = rho.shape[axis]
    return float(np.sum(rho * (np.take(v, np.arange(0, n), axis=axis) + np.take(v, np.arange(1, n + 1), axis=axis))))


def test_transport_moves_energy_and_momenta_without_loss():
    n, dx, mach = 24, 0.05, 0.5
    o = Oracle(n, n, n, dx0=dx, GM=0.0, eps=0.0, L=0.0, noise_amp=0.0, mach=mach, chi=0.0)
    b = _bump(n, 6, 18)
    W = b[None, None, :] * b[None, :, None] * b[:, None, None]
    E0 = o.field(0, "e")[0, 0, 0]
    rng = np.random.default_rng(3)
    o.set_field(0, "rho", 1.0 + 0.05 * W * rng.uniform(0.5, 1.0, W.shape))
    o.set_field(0, "e", E0 * (1.0 + 0.05 * W * rng.uniform(0.5, 1.0, W.shape)))
    shapes = {"vx": (n, n, n + 1), "vy": (n, n + 1, n), "vz": (n + 1, n, n)}
    for name, shp in shapes.items():
        ax = {"vx": 2, "vy": 1, "vz": 0}[name]
        fb = _bump(n + 1, 6, 19)
        wf = np.ones(shp)
        for a2 in range(3):
            prof = fb if a2 == ax else b
            sh = [1, 1, 1]
            sh[a2] = prof.size
            wf = wf * prof.reshape(sh)
        base = -mach if name == "vx" else 0.0
        o.set_full_field(0, name, base + 0.05 * wf * rng.uniform(-1.0, 1.0, shp))
    rho0, e0 = o.field(0, "rho"), o.field(0, "e")
    v0 = {k: o.full_field(0, k) for k in shapes}
    o.stage("transport", 0.02)  # Courant number 0.22
    rho1, e1 = o.field(0, "rho"), o.field(0, "e")
    v1 = {k: o.full_field(0, k) for k in shapes}
    assert not np.array_equal(rho0, rho1)
    assert abs(rho1.sum() - rho0.sum()) <= 1e-13 * rho0.sum()
    assert abs(e1.sum() - e0.sum()) <= 1e-13 * e0.sum()
    for k, ax in (("vx", 2), ("vy", 1), ("vz", 0)):
        # sum of the cell momenta the stage built, against the sum of those it
        # left, read through the rebuilt faces (each interior face holds the
        # two momenta next to it over the two densities next to it)
        before = _cell_momentum(v0[k], rho0, ax)
        after = _face_sum(v1[k], rho1, ax)
        scale = np.sum(np.abs(v0[k])) + 1.0
        assert abs(after - before) <= 1e-13 * scale, (k, before, after)
        assert np.max(np.abs(v1[k] - v0[k])) > 1e-4, k  # the stage did move it
