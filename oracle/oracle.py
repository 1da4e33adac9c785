"""Python handle on the plain FP64 CPU oracle (``oracle/dfo.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  This module only marshals arguments; every step of the method is in the C
file, which follows Sect. 3 of Velasco Romero & Masset (2018).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfo.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIELDS = {"rho": 0, "e": 1, "vx": 2, "vy": 3, "vz": 4}


# -O3 with the x86-64-v3 instruction set (AVX2, FMA) rather than -march=native:
# the library is built on one host and may run on another.  FMA contraction is
# off, and nothing reassociates (no -ffast-math), so the flags change speed
# only, never a result (checked bitwise against an -O2 build by the tests).
OPT_FLAGS = ("-O3", "-march=x86-64-v3")


def build(force: bool = True, path: str = _LIB, opt=OPT_FLAGS) -> str:
    """Compile the oracle with FMA contraction off (plain FP64 arithmetic)."""
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        subprocess.check_call(
            ["gcc", *opt, "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("nlevels", ctypes.c_int), ("g0", ctypes.c_int), ("gf", ctypes.c_int),
        ("dx0", ctypes.c_double), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("rho0", ctypes.c_double), ("cs", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("noise_amp", ctypes.c_double),
        ("GM", ctypes.c_double), ("eps", ctypes.c_double), ("L", ctypes.c_double),
        ("mach", ctypes.c_double), ("chi", ctypes.c_double),
        ("subcycle", ctypes.c_int), ("bcmode", ctypes.c_int), ("visc", ctypes.c_double),
        ("nx1", ctypes.c_int), ("ny1", ctypes.c_int), ("nz1", ctypes.c_int),
        ("quadrant", ctypes.c_int),
    ]


_libs: dict = {}


def _load(path: str = _LIB):
    lib = _libs.get(path)
    if lib is None:
        if not os.path.exists(path):
            build(force=False, path=path)
        lib = ctypes.CDLL(path)
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        lib.dfo_create.restype = vp
        lib.dfo_create.argtypes = [ctypes.POINTER(_Params)]
        lib.dfo_destroy.argtypes = [vp]
        lib.dfo_step.argtypes = [vp, ip]
        lib.dfo_time.restype = ctypes.c_double
        lib.dfo_time.argtypes = [vp]
        lib.dfo_dt.restype = ctypes.c_double
        lib.dfo_dt.argtypes = [vp]
        lib.dfo_force.argtypes = [vp, dp]
        lib.dfo_totals.argtypes = [vp, dp]
        lib.dfo_get_field.argtypes = [vp, ip, ip, dp, ip]
        lib.dfo_set_field.argtypes = [vp, ip, ip, dp, ip]
        lib.dfo_get_lastface.argtypes = [vp, ip, ip, dp]
        lib.dfo_set_lastface.argtypes = [vp, ip, ip, dp]
        lib.dfo_sync.argtypes = [vp]
        lib.dfo_commup.argtypes = [vp, ip]
        lib.dfo_commmean.argtypes = [vp, ip]
        lib.dfo_prolong_all.argtypes = [vp, ip]
        lib.dfo_stage.argtypes = [vp, ip, ctypes.c_double]
        lib.dfo_heat_weights.argtypes = [vp, ip, dp]
        lib.dfo_set_threads.argtypes = [ip]
        lib.dfo_set_threads.restype = None
        lib.dfo_schedule.argtypes = [vp, ctypes.POINTER(ip)]
        lib.dfo_schedule.restype = None
        lib.dfo_choose_schedule.argtypes = [ip, dp, dp, ip, ctypes.POINTER(ip)]
        lib.dfo_choose_schedule.restype = None
        _libs[path] = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One oracle run.  Parameters as in the C ``dfo_params``; field arrays are
    returned with shape (nz, ny, nx) (x fastest), active entries only unless
    ``ghosts=True``."""

    STAGES = {"kick": 1, "compress": 2, "diffuse": 3, "heat": 4, "transport": 5,
              "sources": 6, "level_step": 7, "viscosity": 8}

    def __init__(self, nx, ny=None, nz=None, *, nlevels=1, dx0=None, gamma=5.0 / 3.0,
                 cfl=0.4, rho0=1.0, cs=1.0, seed=1, noise_amp=1e-6, GM=0.01, eps=0.0,
                 L=0.0, mach=0.5, chi=0.1, g0=3, gf=10, threads=None, subcycle=0, bcmode=0, visc=0.0,
                 n1=None, quadrant=False, lib_path=_LIB):
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        if dx0 is None:
            raise ValueError("dx0 is required")
        if threads is not None:
            os.environ["OMP_NUM_THREADS"] = str(threads)
            _load(lib_path).dfo_set_threads(int(threads))
        self._lib = _load(lib_path)
        n1 = tuple(n1) if n1 else (0, 0, 0)
        self.p = _Params(nx, ny, nz, nlevels, g0, gf, dx0, gamma, cfl, rho0, cs, seed,
                         noise_amp, GM, eps, L, mach, chi, int(subcycle), int(bcmode), float(visc),
                         *[int(v) for v in n1], int(bool(quadrant)))
        self.n = (nx, ny, nz)
        # cells of each level (levels >= 1 may be half as wide as level 0)
        self.nl = [self.n] + [(n1 if n1[0] else self.n)] * (nlevels - 1)
        self.nlevels = nlevels
        self.g = [g0] + [gf] * (nlevels - 1)
        self._h = self._lib.dfo_create(ctypes.byref(self.p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.dfo_destroy(h)
            self._h = None

    # --- stepping -------------------------------------------------------
    def step(self, n: int = 1) -> None:
        self._lib.dfo_step(self._h, int(n))

    def stage(self, name: str, dt: float) -> None:
        if self._lib.dfo_stage(self._h, self.STAGES[name], float(dt)) != 0:
            raise ValueError(f"stage {name} not available for this run")

    def dt(self) -> float:
        return self._lib.dfo_dt(self._h)

    def schedule(self) -> list:
        """sub-steps of level l+1 per step of level l in the last coarse step"""
        xi = (ctypes.c_int * max(1, self.nlevels - 1))()
        self._lib.dfo_schedule(self._h, xi)
        return list(xi)[: self.nlevels - 1]

    @property
    def time(self) -> float:
        return self._lib.dfo_time(self._h)

    # --- results ---------------------------------------------------------
    def force(self) -> np.ndarray:
        out = np.zeros(3)
        self._lib.dfo_force(self._h, _dp(out))
        return out

    def totals(self) -> np.ndarray:
        """mass, internal energy, kinetic energy, net boundary mass inflow"""
        out = np.zeros(4)
        self._lib.dfo_totals(self._h, _dp(out))
        return out

    def _shape(self, level, ghosts):
        g = self.g[level] if ghosts else 0
        nx, ny, nz = self.nl[level]
        return (nz + 2 * g, ny + 2 * g, nx + 2 * g)

    def field(self, level: int, name: str, ghosts: bool = False) -> np.ndarray:
        out = np.zeros(self._shape(level, ghosts))
        if self._lib.dfo_get_field(self._h, level, FIELDS[name], _dp(out), int(ghosts)) != 0:
            raise ValueError("bad level/field")
        return out

    def set_field(self, level: int, name: str, arr, ghosts: bool = False) -> None:
        a = np.ascontiguousarray(arr, dtype=np.float64)
        if a.shape != self._shape(level, ghosts):
            raise ValueError(f"shape {a.shape} != {self._shape(level, ghosts)}")
        if self._lib.dfo_set_field(self._h, level, FIELDS[name], _dp(a), int(ghosts)) != 0:
            raise ValueError("bad level/field")

    def last_face(self, level: int, name: str) -> np.ndarray:
        """the face-velocity entries with index n along their own axis"""
        nx, ny, nz = self.nl[level]
        dn = FIELDS[name] - 2
        shp = {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[dn]
        out = np.zeros(shp)
        self._lib.dfo_get_lastface(self._h, level, FIELDS[name], _dp(out))
        return out

    def set_last_face(self, level: int, name: str, arr) -> None:
        a = np.ascontiguousarray(arr, dtype=np.float64)
        self._lib.dfo_set_lastface(self._h, level, FIELDS[name], _dp(a))

    def full_field(self, level: int, name: str) -> np.ndarray:
        """active entries; face fields include entry n along their own axis"""
        a = self.field(level, name)
        if name in ("vx", "vy", "vz"):
            ax = {"vx": 2, "vy": 1, "vz": 0}[name]
            a = np.concatenate([a, np.expand_dims(self.last_face(level, name), ax)], axis=ax)
        return a

    def set_full_field(self, level: int, name: str, arr) -> None:
        a = np.asarray(arr, dtype=np.float64)
        if name in ("vx", "vy", "vz"):
            ax = {"vx": 2, "vy": 1, "vz": 0}[name]
            n = a.shape[ax] - 1
            self.set_field(level, name, np.take(a, np.arange(n), axis=ax))
            self.set_last_face(level, name, np.take(a, n, axis=ax))
        else:
            self.set_field(level, name, a)

    def sync(self) -> None:
        self._lib.dfo_sync(self._h)

    def commup(self, coarse_level: int) -> None:
        self._lib.dfo_commup(self._h, coarse_level)

    def prolong_all(self, coarse_level: int) -> None:
        self._lib.dfo_prolong_all(self._h, coarse_level)

    def commmean(self, coarse_level: int) -> None:
        self._lib.dfo_commmean(self._h, coarse_level)

    def heat_weights(self, level: int) -> np.ndarray:
        nx, ny, nz = self.nl[level]
        out = np.zeros((nz, ny, nx))
        self._lib.dfo_heat_weights(self._h, level, _dp(out))
        return out

    def state(self, level: int = 0, ghosts: bool = False) -> dict:
        return {k: self.field(level, k, ghosts) for k in FIELDS}


def choose_schedule(dtl, cost, use_criterion=True) -> list:
    """App. A: the word xi in {1,2}^(n-1) maximising the coarse step (eq. 55)
    per cost (eq. 56) for per-level limits dtl and per-level-step costs"""
    nl = len(dtl)
    xi = (ctypes.c_int * max(1, nl - 1))()
    a = np.ascontiguousarray(dtl, dtype=np.float64)
    c = np.ascontiguousarray(cost, dtype=np.float64)
    _load().dfo_choose_schedule(nl, _dp(a), _dp(c), int(use_criterion), xi)
    return list(xi)[: nl - 1]
