"""Closed-form linear-theory results quoted by Velasco Romero & Masset (2018).

TEST INFRASTRUCTURE ONLY (used by tests/ to pin the oracle's and the HIP
path's physics).  Each function states the equation it evaluates.  Units:
G = rho0 = c_s = 1 unless the arguments say otherwise.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def plume_length(chi: float, gamma: float, V: float) -> float:
    """Cut-off distance lambda = chi / (gamma V), eq. 7."""
    return chi / (gamma * V)


def response_time(chi: float, gamma: float, V: float) -> float:
    """Settling time tau = lambda^2 / chi = chi / (gamma^2 V^2), eq. 9."""
    return chi / (gamma * gamma * V * V)


def heating_accel_lowmach(gamma, G, L, chi, cs=1.0):
    """Low-Mach heating acceleration, eq. 8 (along the motion)."""
    return gamma * (gamma - 1.0) * G * L / (2.0 * chi * cs * cs)


def heating_density_lowmach(x, y, z, gamma, L, chi, V, cs=1.0):
    """Low-Mach density perturbation of the hot plume, eq. 6 (gas moving along
    +z in that equation's frame)."""
    r = np.sqrt(x * x + y * y + z * z)
    lam = plume_length(chi, gamma, V)
    return -gamma * (gamma - 1.0) * L / (4.0 * math.pi * chi * cs * cs * r) * np.exp((z - r) / (2.0 * lam))


def h_fraction(rp):
    """Fraction of the low-Mach heating force from within r' = r / (2 lambda),
    eq. 23: h = (1 - 2r' - exp(-2r')) / (2 r'^2) + 1."""
    rp = np.asarray(rp, dtype=float)
    return (1.0 - 2.0 * rp - np.exp(-2.0 * rp)) / (2.0 * rp * rp) + 1.0


def mu(u):
    """mu(u) = u exp(-u^2) + (sqrt(pi)/2)(u^-2 - 2) erfc(u), eq. 12."""
    return u * math.exp(-u * u) + 0.5 * math.sqrt(math.pi) * (u ** -2 - 2.0) * special.erfc(u)


def f_highmach(eps: float) -> float:
    """f(eps) = integral_eps^inf mu(sqrt(u)) du, eq. 11."""
    val, _ = integrate.quad(lambda u: mu(math.sqrt(u)), eps, np.inf, limit=400)
    return val


def heating_accel_highmach(gamma, G, L, chi, V, rmin):
    """High-Mach heating acceleration, eq. 10."""
    return 2.0 * (gamma - 1.0) * G * L / (math.sqrt(math.pi) * chi * V * V) * f_highmach(rmin * V / (4.0 * chi))


def heating_increment_per_doubling(gamma, G, M, L, chi, V):
    """Heating-force increment when the finest scale is halved, eq. 24."""
    return (gamma - 1.0) * G * M * L / (chi * V * V) * math.log(2.0)


def cold_integral() -> float:
    """The integral of eq. 47: int_0^inf [-u^{1/2} e^{-u} + (sqrt(pi)/2) erf(u^{1/2})] du / u^2."""
    fun = lambda u: (-math.sqrt(u) * math.exp(-u) + 0.5 * math.sqrt(math.pi) * special.erf(math.sqrt(u))) / (u * u)
    a, _ = integrate.quad(fun, 0.0, 1.0, limit=400)
    b, _ = integrate.quad(fun, 1.0, np.inf, limit=400)
    return a + b


def F0(G, M, rho0=1.0, cs=1.0):
    """Force unit F0 = 4 pi (G M)^2 rho0 / c_s^2, eq. 50."""
    return 4.0 * math.pi * (G * M) ** 2 * rho0 / (cs * cs)


def cold_thermal_force(gamma, G, M, rho0=1.0, cs=1.0):
    """Low-Mach cold thermal force, eqs. 47-48 / 51: -(gamma-1) F0 / 2."""
    return -2.0 * math.pi * G * G * M * M * rho0 * (gamma - 1.0) / (cs * cs)


def critical_luminosity(gamma, G, M, chi, rho0=1.0):
    """L_c = 4 pi G M rho0 chi / gamma, eq. 49."""
    return 4.0 * math.pi * G * M * rho0 * chi / gamma


def heating_force(gamma, G, M, L, chi, rho0=1.0, cs=1.0):
    """Low-Mach heating force, eq. 52: (gamma-1)/2 (L/L_c) F0."""
    return 0.5 * (gamma - 1.0) * L / critical_luminosity(gamma, G, M, chi, rho0) * F0(G, M, rho0, cs)


def thermal_force(gamma, G, M, L, chi, rho0=1.0, cs=1.0):
    """Total low-Mach thermal force, eq. 53."""
    return 0.5 * (gamma - 1.0) * (L / critical_luminosity(gamma, G, M, chi, rho0) - 1.0) * F0(G, M, rho0, cs)
