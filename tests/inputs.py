"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module holds only input recipes: mesh sizes, perturber parameters and
seeded random draws.  It contains none of the method's arithmetic.  Sizing rule
for a run: finest cell = max(lambda / 5, R_B) with lambda = chi / (gamma V) the
plume length (eq. 7) and R_B = G M / c_s^2 the Bondi radius (eq. 17); the
Plummer length (and Gaussian heat width) is two finest cells.
"""
from __future__ import annotations

import numpy as np

GAMMA = 5.0 / 3.0


def finest_dx(mach, chi=0.1, GM=0.01, gamma=GAMMA, cs=1.0):
    V = mach * cs
    lam = chi / (gamma * V)
    return max(lam / 5.0, GM / (cs * cs))


def job(n, nlevels, mach, GM, chi, L, *, seed=1, noise_amp=1e-6, gamma=GAMMA, cfl=0.4,
        dx_finest=None, eps_cells=2.0, n1=None):
    """one run of n^3 cells per level (or n1^3 on the finer levels)"""
    dxf = finest_dx(mach, chi, GM, gamma) if dx_finest is None else dx_finest
    d = dict(nx=n, ny=n, nz=n, nlevels=nlevels, dx0=dxf * 2 ** (nlevels - 1), gamma=gamma,
             cfl=cfl, seed=seed, noise_amp=noise_amp, GM=GM, eps=eps_cells * dxf, L=L,
             mach=mach, chi=chi)
    if n1:
        d["n1"] = (n1, n1, n1)
    return d


def paper_mesh(n0, nlevels, mach, chi, *, GM=1e-3, L=0.0, seed=1, noise_amp=0.0, dx_finest=None):
    """The mesh of the paper's Sects. 4.1.3 and 4.2.2 (its Figs. 8 and 12) with
    the flow along x and the full box standing for the paper's quadrant (x, y
    > 0 there, its mirror images here): a ground level of n0^3 cells and
    finer levels of (n0/2)^3 cells, the first covering the central quarter of
    the ground level, the next ones the central half of the level before;
    gamma 1.4, eps 0, the heat split over the 8 cells around the perturber;
    finest cell lambda / 5 unless given."""
    d = job(n0, nlevels, mach, GM, chi, L, seed=seed, noise_amp=noise_amp, gamma=1.4,
            dx_finest=dx_finest, n1=n0 // 2)
    d["eps"] = 0.0
    return d


def config1():
    """32^3, one level, Mach 0.5, GM 0.01, chi 0.1, L 0, 100 steps, seed 1."""
    return job(32, 1, 0.5, 0.01, 0.1, 0.0, seed=1), 100


def config2(L=1e-3):
    """128^3, one level, Mach 1.5, GM 0.01, chi 0.1, Gaussian heat, 500 steps, seed 2."""
    return job(128, 1, 1.5, 0.01, 0.1, L, seed=2), 500


def config3(L=1e-3, n=128):
    """4 levels of n^3, Mach 0.3, GM 1e-3, chi 0.1, 100 coarse steps, seed 3."""
    return job(n, 4, 0.3, 1e-3, 0.1, L, seed=3), 100


def config4(njobs=64):
    """Batched sweep: edges from {48,64,80,96}, Mach log-uniform [0.1,3],
    L from {0, 1e-3}, GM 0.01, chi 0.1, 200 steps each (rng seed 4)."""
    rng = np.random.default_rng(4)
    jobs = []
    for j in range(njobs):
        n = int(rng.choice([48, 64, 80, 96]))
        mach = float(np.exp(rng.uniform(np.log(0.1), np.log(3.0))))
        L = float(rng.choice([0.0, 1e-3]))
        jobs.append(job(n, 1, mach, 0.01, 0.1, L, seed=1000 + j))
    return jobs, 200


def config5(njobs=400, rate=20.0):
    """Serving: Poisson arrivals (rate jobs/s), edges from {32,48,...,128},
    1-3 levels, Mach log-uniform [0.1,3], L log-uniform [1e-4,1e-2], GM 0.01,
    chi 0.1, 300 coarse steps each (rng seed 5).  Returns (arrival_times, jobs, steps)."""
    rng = np.random.default_rng(5)
    t = np.cumsum(rng.exponential(1.0 / rate, size=njobs))
    jobs = []
    for j in range(njobs):
        n = int(rng.choice(np.arange(32, 129, 16)))
        nl = int(rng.integers(1, 4))
        mach = float(np.exp(rng.uniform(np.log(0.1), np.log(3.0))))
        L = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        jobs.append(job(n, nl, mach, 0.01, 0.1, L, seed=5000 + j))
    return t, jobs, 300


def random_state(shape, seed, *, amp=1e-3, mach=0.5, e0=0.9):
    """A seeded, smooth-ish perturbed state (rho, e, vx, vy, vz) for stage tests."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    e = e0 * (1.0 + amp * rng.uniform(-1, 1, size=shape))
    vx = -mach + amp * rng.uniform(-1, 1, size=shape)
    vy = amp * rng.uniform(-1, 1, size=shape)
    vz = amp * rng.uniform(-1, 1, size=shape)
    return {"rho": rho, "e": e, "vx": vx, "vy": vy, "vz": vz}
