"""Linear-theory pins of the low-Mach forces (Sects. 2.3, 4.1.1, 4.2), run on the
HIP path (which matches the FP64 oracle to 1e-11, tests/test_gpu_parity.py).

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


def _heating_at(dfm, mach, nl, n, dxf, t_end, L=2e-4):
    # hot minus cold force at t_end; both runs share the mesh, so their time
    # steps (diffusion-limited here) and log times coincide
    r = {}
    for lum in (L, 0.0):
        run = dfm.Run(n, nlevels=nl, dx0=dxf * 2 ** (nl - 1), noise_amp=0.0, precision=dfm.DF_FP32)
        run.set_perturber(GM, 0.0, lum, mach, CHI)
        while run.force()[3] < t_end:
            run.step(50)
        log = run.force_log()
        r[lum] = log[int(np.searchsorted(log[:, 3], t_end))]
    assert abs(r[L][3] - r[0.0][3]) < 1e-12 * r[L][3]
    return r[L][0] - r[0.0][0]


def test_high_mach_heating_force_inverse_square(dfm):
    # Sect. 4.1.2: with the mesh fixed in units of lambda (finest cell lambda/5,
    # so r_min V / 4 chi is the same), eq. 10 depends on V only through V^-2
    got = {}
    for mach in (2.0, 3.0):
        lam = CHI / (GAMMA * mach)
        tau = T.response_time(CHI, GAMMA, mach)
        got[mach] = _heating_at(dfm, mach, 3, 48, lam / 5.0, 40 * tau)
    ratio = got[2.0] / got[3.0]
    _say(f"[physics] F_heat(M=2) / F_heat(M=3) = {ratio:.4f} (V^-2 law: 2.25)")
    assert got[3.0] > 0.0 and abs(ratio / 2.25 - 1.0) < 0.05


def test_high_mach_resolution_increment(dfm):
    # Sect. 4.1.2, eq. 24: at Mach 3, adding a finer level (same box, finest
    # cell halved) raises the heating force by (gamma-1) G M L log2 / (chi V^2)
    # in the limit r_min V / 4 chi -> 0; at the finest cells used here (r_min
    # V / 4 chi = 0.015-0.03) eq. 10's f gives 0.80-0.87 of that increment
    mach = 3.0
    lam = CHI / (GAMMA * mach)
    tau = T.response_time(CHI, GAMMA, mach)
    f3 = _heating_at(dfm, mach, 3, 48, lam / 5.0, 40 * tau)
    f4 = _heating_at(dfm, mach, 4, 48, lam / 10.0, 40 * tau)
    inc = T.heating_increment_per_doubling(GAMMA, 1.0, GM, 2e-4, CHI, mach)
    _say(f"[physics] Mach 3 increment {f4 - f3:.4e} vs eq. 24 {inc:.4e} (ratio {(f4 - f3) / inc:.3f})")
    assert 0.72 < (f4 - f3) / inc < 0.97
