"""Pins of the closed-form linear-theory module against the numbers the paper
prints (Sects. 4.1.1, 4.2.2, 4.3.2) and against the paper's own algebra."""
import json
import math
import os

import numpy as np
import pytest

from oracle import theory as T

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_fig6_fraction():
    # Sect. 4.1.1: finest cell 25/128 lambda -> r'_min = 25/256, r'_max = 50: "about 92%"
    g = GOLD["fig6_low_mach_fraction"]
    frac = T.h_fraction(50.0) - T.h_fraction(25.0 / 256.0)
    assert abs(frac - g["value"]) < g["tol"]


def test_fig12_fractions():
    # Sect. 4.2.2: box l = 3200 lambda for chi = 0.1, ground 64 cells over l, first
    # level a quarter of it with 32 cells, 11 levels in all -> finest dx = l / 131072.
    # The box is fixed in absolute units, so for chi = 0.05, 0.01 the scaled
    # r' grow as 0.1 / chi.  The paper prints 99.1 %, 98.4 %, 92.3 %.
    g = GOLD["fig12_fractions"]
    for chis, want in g["value"].items():
        chi = float(chis)
        s = 0.1 / chi
        rmax = 1600.0 * s
        rmin = (3200.0 / 131072.0) / 2.0 * s
        frac = float(T.h_fraction(rmax) - T.h_fraction(rmin))
        assert abs(frac - want) < g["tol"], (chi, frac)


def test_fig14_fraction():
    # Sect. 4.3.2: r'_min = 0.01, r'_max = 1600 retrieve "99%" of the heating force
    g = GOLD["fig14_fraction"]
    frac = float(T.h_fraction(1600.0) - T.h_fraction(0.01))
    assert abs(frac - g["value"]) < g["tol"]


def test_h_limits():
    # h -> 0 as r' -> 0 (no material inside) and -> 1 as r' -> inf (eq. 23)
    assert abs(float(T.h_fraction(1e-4))) < 1e-3
    assert abs(float(T.h_fraction(1e6)) - 1.0) < 1e-5


def test_cold_integral_is_sqrt_pi():
    # eq. 47: the prefactor -2 pi^{1/2} G^2 M^2 rho0 (gamma-1)/c^2 times the
    # integral equals -2 pi G^2 M^2 rho0 (gamma-1)/c^2, so the integral is sqrt(pi)
    assert abs(T.cold_integral() - math.sqrt(math.pi)) < 1e-8


def test_small_eps_constant():
    # eqs. 10 and 13: (2/sqrt(pi)) f(eps) ~ -1.96 - log(eps) for small eps
    for eps in (1e-8, 1e-10):
        c = 2.0 / math.sqrt(math.pi) * T.f_highmach(eps) + math.log(eps)
        assert abs(c - GOLD["eq13_constant"]["value"]) < GOLD["eq13_constant"]["tol"], (eps, c)


def test_critical_luminosity_balances_cold_force():
    # eq. 49 is obtained by equating eq. 8 (times M) with minus eq. 48
    for gamma in (1.4, 5.0 / 3.0):
        GM, chi = 1e-3, 0.1
        Lc = T.critical_luminosity(gamma, 1.0, GM, chi)
        heat = GM * T.heating_accel_lowmach(gamma, 1.0, Lc, chi)
        assert abs(heat + T.cold_thermal_force(gamma, 1.0, GM)) < 1e-15
        assert abs(T.thermal_force(gamma, 1.0, GM, Lc, chi)) < 1e-15


def test_cold_force_minus_point_two():
    # Fig. 12 caption: at gamma = 1.4 the normalised cold force tends to -0.2
    F = T.cold_thermal_force(1.4, 1.0, 1e-3) / T.F0(1.0, 1e-3)
    assert abs(F - GOLD["cold_force_gamma14"]["value"]) < GOLD["cold_force_gamma14"]["tol"]


def test_heating_force_normalised():
    # eq. 52 equals M times eq. 8
    gamma, GM, L, chi = 5.0 / 3.0, 1e-3, 2e-4, 0.1
    assert math.isclose(T.heating_force(gamma, 1.0, GM, L, chi),
                        GM * T.heating_accel_lowmach(gamma, 1.0, L, chi), rel_tol=1e-14)


def test_plume_profile_scale():
    # eq. 6 along the downstream axis (z > 0 in that frame): pure 1/r law
    gamma, L, chi, V = 5.0 / 3.0, 1e-3, 0.1, 0.1
    z = np.array([0.5, 1.0, 2.0])
    rho = T.heating_density_lowmach(0 * z, 0 * z, z, gamma, L, chi, V)
    assert np.allclose(rho * z, rho[0] * z[0], rtol=1e-14)
    # upstream the cut-off length is lambda: exp(-r/lambda) factor
    lam = T.plume_length(chi, gamma, V)
    up = T.heating_density_lowmach(0.0, 0.0, -lam, gamma, L, chi, V)
    dn = T.heating_density_lowmach(0.0, 0.0, lam, gamma, L, chi, V)
    assert math.isclose(up / dn, math.exp(-1.0), rel_tol=1e-14)
