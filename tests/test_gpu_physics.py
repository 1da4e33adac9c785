"""Linear-theory pins of the forces (Sects. 2.3, 4.1, 4.2), run on the HIP path
(which matches the FP64 oracle to 1e-11, tests/test_gpu_parity.py): single
points at gamma 5/3 on the central-half hierarchy, and the sweeps of the
paper's Figs. 6, 9 and 12 in its own setup and on its own meshes (below).

Setup as in the paper: perturber on the central vertex, epsilon = 0, heat split
over the 8 cells around it, finest cell lambda/5 (r'_min = 0.1), GM / (chi c_s)
= 0.01 (linear regime), gamma = 5/3.  The forces are differences of two runs
(eq. 5): the heating force F(M,L,chi) - F(M,0,chi), the cold thermal force
F(M,0,chi) - F(M,0,0).  Expected values are the closed forms of eq. 8 (times
the perturber mass) and eq. 51, scaled by the finite-range fraction
h(r'_max) - h(r'_min) of eq. 23."""
import sys

import numpy as np
import pytest

from oracle import theory as T

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0
CHI = 0.1
GM = 1e-3


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


def _force_at(dfm, mach, nlevels, n, L, chi, t_end, gamma=GAMMA, walls=False):
    lam = CHI / (gamma * mach)
    dxf = lam / 5.0
    r = dfm.Run(n, nlevels=nlevels, dx0=dxf * 2 ** (nlevels - 1), gamma=gamma, noise_amp=0.0,
                precision=dfm.DF_FP32)
    if walls:
        r.set_boundaries(1)
    r.set_perturber(GM, 0.0, L, mach, chi)
    while True:
        r.step(50)
        f = r.force()
        if f[3] >= t_end:
            break
    log = r.force_log()
    k = int(np.searchsorted(log[:, 3], t_end))
    return log[min(k, len(log) - 1)]


def _fraction(mach, nlevels, n, gamma=GAMMA):
    lam = CHI / (gamma * mach)
    dxf = lam / 5.0
    rmax = (n // 2) * dxf * 2 ** (nlevels - 1) / (2 * lam)
    return float(T.h_fraction(rmax) - T.h_fraction(dxf / (2 * lam)))


LOW = dict(mach=0.1, nl=5, n=64, L=2e-4)


@pytest.fixture(scope="module")
def low_mach_pair(dfm):
    # Mach 0.1, L = 2e-4 (Sect. 4.1), 5 levels of 64^3 (r' from 0.1 to 51.2):
    # the hot and the cold run at 50 tau, force logs and finest-level densities
    mach, nl, n = LOW["mach"], LOW["nl"], LOW["n"]
    lam = CHI / (GAMMA * mach)
    tau = T.response_time(CHI, GAMMA, mach)
    out = {}
    for lum in (LOW["L"], 0.0):
        r = dfm.Run(n, nlevels=nl, dx0=lam / 5.0 * 2 ** (nl - 1), noise_amp=0.0, precision=dfm.DF_FP32)
        r.set_perturber(GM, 0.0, lum, mach, CHI)
        while r.force()[3] < 50 * tau:
            r.step(50)
        log = r.force_log()
        out[lum] = (log[min(int(np.searchsorted(log[:, 3], 50 * tau)), len(log) - 1)], r.field(nl - 1, "rho"))
    return out


def test_low_mach_heating_force(dfm, low_mach_pair):
    # after 50 tau the heating force is within 5 % of M a(eq. 8) (h(r'max) - h(r'min))
    hot, cold = low_mach_pair[LOW["L"]][0], low_mach_pair[0.0][0]
    want = GM * T.heating_accel_lowmach(GAMMA, 1.0, LOW["L"], CHI) * _fraction(LOW["mach"], LOW["nl"], LOW["n"])
    got = hot[0] - cold[0]
    _say(f"[physics] heating force {got:.5e} vs {want:.5e} (ratio {got / want:.4f})")
    assert got > 0.0
    assert abs(got / want - 1.0) < 0.05


def test_low_mach_density_profile_cuts(dfm, low_mach_pair):
    # Sect. 4.1.1, Fig. 8: the hot-minus-cold density on the finest level along
    # the flow axis and across it follows eq. 6: an inverse law downstream, a
    # cut-off exp(-r / lambda) upstream and exp(-r / 2 lambda) transversally.
    # The gas moves along -x here (eq. 6's z is -x); each cut averages the four
    # cells around its axis and eq. 6 is averaged over the same four centres.
    mach, nl, n, L = LOW["mach"], LOW["nl"], LOW["n"], LOW["L"]
    lam = CHI / (GAMMA * mach)
    dx = lam / 5.0
    d = low_mach_pair[L][1] - low_mach_pair[0.0][1]  # (z, y, x)
    c = n // 2
    xs = (np.arange(n) - n / 2 + 0.5) * dx
    h = dx / 2

    def eq6(x, y, z):  # our coordinates; eq. 6's z axis is -x
        return T.heating_density_lowmach(y, z, -x, GAMMA, L, CHI, mach)

    worst = {"downstream": 0.0, "upstream": 0.0, "transverse": 0.0}
    for i in range(n):
        x = xs[i]
        got = 0.25 * (d[c - 1, c - 1, i] + d[c - 1, c, i] + d[c, c - 1, i] + d[c, c, i])
        want = eq6(x, h, h)
        if -4.8 * lam < x < -1.4 * lam:
            worst["downstream"] = max(worst["downstream"], abs(got / want - 1.0))
        if 0.8 * lam < x < 2.0 * lam:
            worst["upstream"] = max(worst["upstream"], abs(got / want - 1.0))
    for j in range(c, n):
        y = xs[j]
        got = 0.25 * (d[c - 1, j, c - 1] + d[c - 1, j, c] + d[c, j, c - 1] + d[c, j, c])
        want = 0.5 * (eq6(-h, y, h) + eq6(h, y, h))
        if 0.8 * lam < y < 5.0 * lam:
            worst["transverse"] = max(worst["transverse"], abs(got / want - 1.0))
    _say(f"[physics] eq. 6 cuts, largest relative deviation {worst}")
    assert worst["downstream"] < 0.01 and worst["upstream"] < 0.035 and worst["transverse"] < 0.03, worst


def test_low_mach_cold_thermal_force(dfm):
    # Mach 0.2, 6 levels of 64^3 (r'_max 102): the acoustic sphere reaches the
    # box edge only after ~68 tau, so at 40 tau the cold thermal force is free
    # of reflections (Sect. 4.2.2); it tends to -(gamma-1)/2 F0 (eq. 51)
    mach, nl, n = 0.2, 6, 64
    tau = T.response_time(CHI, GAMMA, mach)
    diff = _force_at(dfm, mach, nl, n, 0.0, CHI, 40 * tau)
    adi = _force_at(dfm, mach, nl, n, 0.0, 0.0, 40 * tau)
    want = T.cold_thermal_force(GAMMA, 1.0, GM) * _fraction(mach, nl, n)
    got = diff[0] - adi[0]
    _say(f"[physics] cold thermal force {got:.5e} vs {want:.5e} (ratio {got / want:.4f})")
    assert got < 0.0
    assert abs(got / want - 1.0) < 0.08


def test_paper_setup_cold_thermal_force(dfm):
    # the paper's own setup (Sect. 3.4): gamma 1.4, eps 0, heat split over the
    # 8 cells, background state at both flow ends and mirror walls; at Mach
    # 0.2 (6 levels of 64^3, 40 tau, before the acoustic sphere reaches the
    # box) the cold thermal force tends to -(gamma-1)/2 F0 = -0.2 F0 (eq. 51,
    # Fig. 12) times the h-fraction of the finite range
    mach, nl, n, gamma = 0.2, 6, 64, 1.4
    tau = T.response_time(CHI, gamma, mach)
    diff = _force_at(dfm, mach, nl, n, 0.0, CHI, 40 * tau, gamma=gamma, walls=True)
    adi = _force_at(dfm, mach, nl, n, 0.0, 0.0, 40 * tau, gamma=gamma, walls=True)
    F0 = T.F0(1.0, GM)
    want = T.cold_thermal_force(gamma, 1.0, GM) * _fraction(mach, nl, n, gamma)
    got = diff[0] - adi[0]
    _say(f"[physics] paper setup: cold thermal force {got / F0:.4f} F0 vs {want / F0:.4f} F0 (ratio {got / want:.4f})")
    assert abs(T.cold_thermal_force(gamma, 1.0, GM) / F0 + 0.2) < 1e-12
    assert got < 0.0
    assert abs(got / want - 1.0) < 0.08


# ---------------------------------------------------- sweeps on the paper's meshes
#
# The paper's own setup (Sect. 3.4: gamma 1.4, eps 0, heat split over the 8
# cells around the perturber, background state at both flow ends, mirror
# walls), with the flow along x and the full box standing for the paper's
# quadrant (its mirror images).  Fig. 6 and Fig. 9 use the mesh of Sect. 4.1:
# 6 levels of 16 x 16 x 32 (here 32^3 per level, each covering the central half
# of the one below), finest cell 25/128 lambda; Fig. 12 the mesh of Sect.
# 4.2.2 at reduced depth: a ground level of 64 x 64 x 128 and finer levels of
# 32 x 32 x 64 (here 64^3 and 32^3), the first covering the central quarter.

PG = 1.4  # gamma of the paper's setup
LUM = 2e-4


def _paper_force(dfm, mach, nl, n, dxf, L, chi, t_end, n1=None):
    r = dfm.Run(n, nlevels=nl, dx0=dxf * 2 ** (nl - 1), gamma=PG, noise_amp=0.0, precision=dfm.DF_FP32,
                n1=n1)
    r.set_boundaries(1)
    r.set_perturber(GM, 0.0, L, mach, chi)
    while r.force()[3] < t_end:
        r.step(50)
    log = r.force_log()
    k = int(np.searchsorted(log[:, 3], t_end))
    return log[min(k, len(log) - 1)]


def _paper_heating(dfm, mach, nl, dxf, t_end):
    # hot minus cold force at t_end (both runs share the mesh and time steps)
    hot = _paper_force(dfm, mach, nl, 32, dxf, LUM, CHI, t_end)
    cold = _paper_force(dfm, mach, nl, 32, dxf, 0.0, CHI, t_end)
    assert abs(hot[3] - cold[3]) < 1e-12 * hot[3]
    return hot[0] - cold[0]


FIG6_MACH = (0.1, 0.2, 0.4, 1.0, 2.0, 3.0)


@pytest.fixture(scope="module")
def fig6(dfm):
    # heating force at 50 tau (40 tau above Mach 1) for each Mach number, on the
    # Fig. 6 mesh: l = 100 lambda, r'_max = 50, r'_min = 25/256
    out = {}
    for mach in FIG6_MACH:
        lam = CHI / (PG * mach)
        tau = T.response_time(CHI, PG, mach)
        out[mach] = _paper_heating(dfm, mach, 6, 25.0 / 128.0 * lam, (50 if mach < 1 else 40) * tau)
        _say(f"[fig6] Mach {mach}: heating force {out[mach]:.5e}")
    return out


def _fig6_plateau():
    dxf_over_lam = 25.0 / 128.0
    h = float(T.h_fraction(16 * dxf_over_lam * 32 / 2) - T.h_fraction(dxf_over_lam / 2))
    return GM * T.heating_accel_lowmach(PG, 1.0, LUM, CHI) * h, h


def test_fig6_low_mach_plateau(fig6):
    # eq. 8 times the perturber's mass and the fraction h(50) - h(25/256) = 0.92
    # (Sect. 4.1.1; the paper finds its low-Mach points within ~3 %)
    want, h = _fig6_plateau()
    assert abs(h - 0.918) < 1e-3
    for mach in (0.1, 0.2):
        _say(f"[fig6] Mach {mach}: {fig6[mach] / want:.4f} of eq. 8 x h")
        assert abs(fig6[mach] / want - 1.0) < 0.05, mach


def test_fig6_transonic_rise(fig6):
    # the force rises from the plateau to a peak at the transonic point
    # (Sect. 4.1.3: eq. 25's ratio exceeds one when the plume is resolved);
    # it is positive everywhere
    want, _ = _fig6_plateau()
    assert all(f > 0.0 for f in fig6.values())
    assert fig6[0.2] < fig6[0.4] < fig6[1.0]
    assert fig6[1.0] == max(fig6.values())
    xi = 4.0 / (np.sqrt(np.pi) * PG) * T.f_highmach(25.0 / 128.0 * (CHI / PG) / (4.0 * CHI))
    _say(f"[fig6] transonic / plateau {fig6[1.0] / want:.3f} (eq. 25 with r_min one finest cell: {xi:.3f})")
    assert fig6[1.0] / want > 1.5


def test_fig6_supersonic_tail(fig6):
    # eq. 10 with the mesh fixed in units of lambda: F proportional to V^-2
    # (Sect. 4.1.2), so F M^2 is the same at Mach 2 and 3
    a, b = fig6[2.0] * 4.0, fig6[3.0] * 9.0
    _say(f"[fig6] F M^2 at Mach 2 and 3: {a:.4e}, {b:.4e} (ratio {a / b:.4f})")
    assert abs(a / b - 1.0) < 0.05


def test_fig9_resolution_increments(dfm):
    # Sect. 4.1.2, eq. 24: at Mach 3 each added finer level (same ground, the
    # finest cell halved) raises the heating force by (gamma-1) G M L log 2 /
    # (chi V^2) in the limit r_min V / 4 chi -> 0; at the finest cells used
    # here (r_min V / 4 chi = 0.14, 0.07, 0.035) the increments approach it from
    # below
    mach = 3.0
    lam = CHI / (PG * mach)
    tau = T.response_time(CHI, PG, mach)
    F = {nl: _paper_heating(dfm, mach, nl, 25.0 / 128.0 * lam * 2 ** (6 - nl), 40 * tau) for nl in (4, 5, 6)}
    inc = T.heating_increment_per_doubling(PG, 1.0, GM, LUM, CHI, mach)
    r1, r2 = (F[5] - F[4]) / inc, (F[6] - F[5]) / inc
    _say(f"[fig9] Mach 3 increments: {r1:.3f}, {r2:.3f} of eq. 24")
    assert 0.7 < r1 < 1.0 and 0.7 < r2 < 1.0
    assert r2 > r1


FIG12_CHI = (0.1, 0.05, 0.01)


def test_fig12_cold_thermal_force_chi_sweep(dfm):
    # Sect. 4.2.2, Fig. 12: the cold thermal force F(M,0,chi) - F(M,0,0) tends
    # to -(gamma-1)/2 F0 = -0.2 F0 (eq. 51) whatever chi, times the fraction of
    # the finite range (the paper assumes eq. 23's); Mach 0.2, 40 tau, each chi
    # on its own mesh in units of lambda (finest cell lambda / 5, r'_max 102,
    # 6 levels: ground 64^3, finer levels 32^3, the first covering the central
    # quarter), so that the acoustic sphere stays inside the box (it reaches
    # 0.7 of the ground level's half-width); GM / chi rises to 0.1 at chi = 0.01,
    # where the flow near the perturber starts to be non-linear
    mach, nl, n0 = 0.2, 6, 64
    F0 = T.F0(1.0, GM)
    got = {}
    for chi in FIG12_CHI:
        lam = chi / (PG * mach)
        dxf = lam / 5.0
        tau = T.response_time(chi, PG, mach)
        diff = _paper_force(dfm, mach, nl, n0, dxf, 0.0, chi, 40 * tau, n1=(32, 32, 32))
        adi = _paper_force(dfm, mach, nl, n0, dxf, 0.0, 0.0, 40 * tau, n1=(32, 32, 32))
        rmax = (n0 // 2) * dxf * 2 ** (nl - 1) / (2 * lam)
        h = float(T.h_fraction(rmax) - T.h_fraction(dxf / (2 * lam)))
        want = T.cold_thermal_force(PG, 1.0, GM) * h
        got[chi] = (diff[0] - adi[0]) / want
        _say(f"[fig12] chi {chi}: cold thermal force {(diff[0] - adi[0]) / F0:.4f} F0, {got[chi]:.4f} of eq. 51 x h")
    assert abs(T.cold_thermal_force(PG, 1.0, GM) / F0 + 0.2) < 1e-12
    for chi in (0.1, 0.05):
        assert abs(got[chi] - 1.0) < 0.05, chi
    assert abs(got[0.01] - 1.0) < 0.08


def test_fig12_on_the_papers_quadrant_mesh(dfm):
    # Sect. 4.2.2's mesh itself: the quadrant bounded by the mirror planes
    # (here y, z > 0 with the flow along x), a ground level of 64 x 64 x 128
    # cells (128 along the flow) and finer levels of 32 x 32 x 64, the first
    # covering the quarter next to the planes, at reduced depth (6 levels,
    # finest cell lambda / 5); chi 0.1, Mach 0.2, 40 tau: the cold thermal
    # force of the whole gas against eq. 51 x h, the range running to the
    # ground level's extent from the planes
    mach, nl, chi = 0.2, 6, 0.1
    lam = chi / (PG * mach)
    dxf = lam / 5.0
    tau = T.response_time(chi, PG, mach)

    def run(c):
        r = dfm.Run(128, 64, 64, nlevels=nl, dx0=dxf * 2 ** (nl - 1), gamma=PG, noise_amp=0.0,
                    precision=dfm.DF_FP32, n1=(64, 32, 32), quadrant=True)
        r.set_boundaries(1)
        r.set_perturber(GM, 0.0, 0.0, mach, c)
        while r.force()[3] < 40 * tau:
            r.step(50)
        log = r.force_log()
        return log[min(int(np.searchsorted(log[:, 3], 40 * tau)), len(log) - 1)]

    diff, adi = run(chi), run(0.0)
    assert diff[1] == 0.0 and diff[2] == 0.0  # the mirror images cancel them
    rmax = 64 * dxf * 2 ** (nl - 1) / (2 * lam)
    h = float(T.h_fraction(rmax) - T.h_fraction(dxf / (2 * lam)))
    want = T.cold_thermal_force(PG, 1.0, GM) * h
    ratio = (diff[0] - adi[0]) / want
    _say(f"[fig12] paper's quadrant mesh, chi {chi}: {(diff[0] - adi[0]) / T.F0(1.0, GM):.4f} F0, "
         f"{ratio:.4f} of eq. 51 x h (h = {h:.4f})")
    assert abs(ratio - 1.0) < 0.05
