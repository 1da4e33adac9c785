"""ctypes marshalling for libdfmesh.so.  One Python function per C entry point
(same names without the ``df_`` prefix) plus :class:`Run`, which owns a
device arena allocated by PyTorch and binds the current HIP stream."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdfmesh.so")

DF_FP64, DF_FP32 = 0, 1
FIELDS = {"rho": 0, "e": 1, "vx": 2, "vy": 3, "vz": 4}
STAGES = {"kick": 1, "compress": 2, "diffuse": 3, "heat": 4, "transport": 5, "sources": 6,
          "level_step": 7, "viscosity": 8}


class DFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdfmesh error {code}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nlevels", ctypes.c_int32),
        ("dx0", ctypes.c_double), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("precision", ctypes.c_int32), ("ghost_fine", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("noise_amp", ctypes.c_double),
        ("tile_chunk", ctypes.c_int32),
        ("nx1", ctypes.c_int32), ("ny1", ctypes.c_int32), ("nz1", ctypes.c_int32),
        ("quadrant", ctypes.c_int32),
    ]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is not built; run paper_1812_03191_amd/build.py (there is no CPU fallback)")
    # the HIP runtime that PyTorch loaded must be the one the library uses
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    sig = {
        "df_init_mesh": [ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)],
        "df_required_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "df_bind": [vp, vp, ctypes.c_size_t, vp],
        "df_set_perturber": [vp] + [ctypes.c_double] * 5,
        "df_step": [vp, i32],
        "df_force": [vp, dp],
        "df_totals": [vp, dp],
        "df_get_field": [vp, i32, i32, dp],
        "df_set_field": [vp, i32, i32, dp],
        "df_sync_levels": [vp],
        "df_get_dt": [vp, dp],
        "df_debug_stage": [vp, i32, ctypes.c_double],
        "df_destroy": [vp],
        "df_force_log": [vp, dp, i32, ctypes.POINTER(i32)],
        "df_timing_enable": [vp, i32],
        "df_timing_read": [vp, dp, ctypes.POINTER(i32), i32],
        "df_stream_copy": [vp, vp, ctypes.c_size_t, vp],
        "df_set_subcycling": [vp, i32],
        "df_set_boundaries": [vp, i32],
        "df_set_transport_fusion": [vp, i32],
        "df_set_kick_fusion": [vp, i32],
        "df_set_finish_fusion": [vp, i32],
        "df_set_step_graphs": [vp, i32],
        "df_set_viscosity": [vp, ctypes.c_double],
        "df_get_schedule": [vp, ctypes.POINTER(i32), i32],
        "df_force_density": [vp, i32, i32, i32] + [ctypes.c_double] * 4 + [vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.df_strerror.restype = ctypes.c_char_p
    lib.df_strerror.argtypes = [ctypes.c_int]
    lib.df_last_error.restype = ctypes.c_char_p
    lib.df_last_error.argtypes = []
    _lib = lib
    return lib


def _ck(rc: int) -> None:
    if rc != 0:
        raise DFError(rc, _lib.df_last_error().decode() or _lib.df_strerror(rc).decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------- entry points

def mesh_desc(nx, ny, nz, nlevels, dx0, gamma=5.0 / 3.0, cfl=0.4, precision=DF_FP64,
              ghost_fine=0, seed=1, noise_amp=1e-6, tile_chunk=0, n1=None, quadrant=False) -> MeshDesc:
    n1 = tuple(n1) if n1 else (0, 0, 0)
    return MeshDesc(nx, ny, nz, nlevels, dx0, gamma, cfl, precision, ghost_fine, seed, noise_amp,
                    tile_chunk, *[int(v) for v in n1], int(quadrant))


def init_mesh(nx, ny, nz, nlevels, dx0, gamma=5.0 / 3.0, cfl=0.4, precision=DF_FP64,
              ghost_fine=0, seed=1, noise_amp=1e-6, tile_chunk=0, n1=None, quadrant=False) -> int:
    lib = _load()
    d = mesh_desc(nx, ny, nz, nlevels, dx0, gamma, cfl, precision, ghost_fine, seed, noise_amp,
                  tile_chunk, n1, quadrant)
    h = ctypes.c_void_p()
    _ck(lib.df_init_mesh(ctypes.byref(d), ctypes.byref(h)))
    return h.value


def required_bytes(h) -> int:
    n = ctypes.c_size_t()
    _ck(_load().df_required_bytes(h, ctypes.byref(n)))
    return n.value


def bind(h, dev_ptr: int, nbytes: int, stream: int) -> None:
    _ck(_load().df_bind(h, dev_ptr, nbytes, stream))


def set_perturber(h, GM, eps, L, mach, chi) -> None:
    _ck(_load().df_set_perturber(h, GM, eps, L, mach, chi))


def step(h, n: int) -> None:
    _ck(_load().df_step(h, int(n)))


def force(h) -> np.ndarray:
    out = np.zeros(4)
    _ck(_load().df_force(h, _dp(out)))
    return out


def totals(h) -> np.ndarray:
    out = np.zeros(3)
    _ck(_load().df_totals(h, _dp(out)))
    return out


def get_field(h, level: int, field: int, out: np.ndarray) -> None:
    _ck(_load().df_get_field(h, level, field, _dp(out)))


def set_field(h, level: int, field: int, arr: np.ndarray) -> None:
    _ck(_load().df_set_field(h, level, field, _dp(arr)))


def sync_levels(h) -> None:
    _ck(_load().df_sync_levels(h))


def get_dt(h) -> float:
    out = ctypes.c_double()
    _ck(_load().df_get_dt(h, ctypes.byref(out)))
    return out.value


def debug_stage(h, stage: int, dt: float) -> None:
    _ck(_load().df_debug_stage(h, int(stage), float(dt)))


def destroy(h) -> None:
    _ck(_load().df_destroy(h))


def force_log(h, cap: int = 4096) -> np.ndarray:
    out = np.zeros((cap, 4))
    n = ctypes.c_int32()
    _ck(_load().df_force_log(h, _dp(out), cap, ctypes.byref(n)))
    return out[: n.value].copy()


KERNEL_KINDS = ("kick", "compress", "diffuse_heat", "pass_x", "pass_y", "pass_z", "rebuild_kick",
                "commup", "commmean", "dt", "force", "zero", "viscosity", "pass_xy", "kick_compress",
                "pass_z_finish")


def timing_enable(h, max_launches: int) -> None:
    _ck(_load().df_timing_enable(h, int(max_launches)))


def timing_read(h) -> dict:
    nk = len(KERNEL_KINDS)
    ms = np.zeros(nk)
    cnt = (ctypes.c_int32 * nk)()
    _ck(_load().df_timing_read(h, _dp(ms), cnt, nk))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}


def stream_copy(dst, src, stream=None) -> None:
    """plain device copy (measurement reference) between two torch tensors of
    the same byte size, 16-byte aligned, on `stream` (default: the current)"""
    import torch

    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("sizes differ")
    st = stream if stream is not None else torch.cuda.current_stream()
    _ck(_load().df_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, st.cuda_stream))


def force_density(rho, dx, GM, eps, rho0=1.0, out=None, stream=None):
    """eq. 18 over one level's density field with no device allocation
    (df_force_density): rho a contiguous float64 CUDA tensor of shape
    (nz, ny, nx); out a float64 CUDA tensor of 3 entries (made if None);
    asynchronous on `stream` (default: the current).  Returns out."""
    import torch

    if rho.dtype != torch.float64 or not rho.is_cuda or not rho.is_contiguous() or rho.dim() != 3:
        raise ValueError("rho must be a contiguous 3-D float64 CUDA tensor")
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=rho.device)
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 3:
        raise ValueError("out must be a float64 CUDA tensor of 3 entries")
    st = stream if stream is not None else torch.cuda.current_stream(rho.device)
    nz, ny, nx = rho.shape
    _ck(_load().df_force_density(rho.data_ptr(), nx, ny, nz, float(dx), float(GM), float(eps), float(rho0),
                                 out.data_ptr(), st.cuda_stream))
    return out


# ------------------------------------------------------------------ Run

class Run:
    """One solver run on a GPU: the arena is a uint8 torch tensor on
    ``device``; kernels go to the stream current at construction."""

    def __init__(self, nx, ny=None, nz=None, *, nlevels=1, dx0, gamma=5.0 / 3.0, cfl=0.4,
                 precision=DF_FP64, ghost_fine=0, seed=1, noise_amp=1e-6, tile_chunk=0,
                 n1=None, quadrant=False, device="cuda"):
        import torch

        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.n = (nx, ny, nz)
        self.nlevels = nlevels
        # cells of each level (the finer levels may have their own, n1)
        self.nl = [self.n] + [tuple(n1) if n1 else self.n] * (nlevels - 1)
        self._h = init_mesh(nx, ny, nz, nlevels, dx0, gamma, cfl, precision, ghost_fine, seed,
                            noise_amp, tile_chunk, n1, quadrant)
        self.nbytes = required_bytes(self._h)
        self.device = torch.device(device)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        bind(self._h, self.arena.data_ptr(), self.nbytes, self.stream.cuda_stream)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                destroy(h)
            finally:
                self._h = None

    @property
    def handle(self):
        return self._h

    def set_perturber(self, GM, eps, L, mach, chi):
        set_perturber(self._h, GM, eps, L, mach, chi)

    def step(self, n=1):
        step(self._h, n)

    def force(self):
        return force(self._h)

    def totals(self):
        return totals(self._h)

    def dt(self):
        return get_dt(self._h)

    def set_subcycling(self, mode: int) -> None:
        """0: two sub-steps per level; 1: the criterion of App. A each coarse step"""
        _ck(_load().df_set_subcycling(self._h, int(mode)))

    def set_viscosity(self, c2: float) -> None:
        """artificial-viscosity coefficient (0: off)"""
        _ck(_load().df_set_viscosity(self._h, float(c2)))

    def set_boundaries(self, mode: int) -> None:
        """0: inflow at x_max, outflow elsewhere; 1: the boundary list of Sect. 3.4"""
        _ck(_load().df_set_boundaries(self._h, int(mode)))

    def set_transport_fusion(self, on: bool) -> None:
        """fuse the x and y transport passes of level 0 and of the finer levels where they qualify (default on)"""
        _ck(_load().df_set_transport_fusion(self._h, int(bool(on))))

    def set_kick_fusion(self, on: bool) -> None:
        """kick and compress in one launch where it qualifies: level 0, and the finer levels in FP32 (default on)"""
        _ck(_load().df_set_kick_fusion(self._h, int(bool(on))))

    def set_finish_fusion(self, on: bool) -> None:
        """fuse a single-level step's z pass with the rebuild and kick where it qualifies (default on)"""
        _ck(_load().df_set_finish_fusion(self._h, int(bool(on))))

    def set_step_graphs(self, on: bool) -> None:
        """replay HIP graphs of two coarse steps in step() on nested runs (default on)"""
        _ck(_load().df_set_step_graphs(self._h, int(bool(on))))

    def schedule(self) -> list:
        """sub-steps of level l+1 per step of level l in the last coarse step"""
        n = max(1, self.nlevels - 1)
        xi = (ctypes.c_int32 * n)()
        _ck(_load().df_get_schedule(self._h, xi, n))
        return list(xi)[: self.nlevels - 1]

    def force_log(self, cap=4096):
        return force_log(self._h, cap)

    def sync_levels(self):
        sync_levels(self._h)

    def stage(self, name, dt):
        debug_stage(self._h, STAGES[name], dt)

    def shape(self, name, level=0):
        nx, ny, nz = self.nl[level]
        e = [nx, ny, nz]
        if name in ("vx", "vy", "vz"):
            e["xyz".index(name[1])] += 1
        return (e[2], e[1], e[0])

    def field(self, level, name):
        out = np.zeros(self.shape(name, level))
        get_field(self._h, level, FIELDS[name], out)
        return out

    def set_field(self, level, name, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        if a.shape != self.shape(name, level):
            raise ValueError(f"shape {a.shape} != {self.shape(name, level)}")
        set_field(self._h, level, FIELDS[name], a)


# ------------------------------------------------------------------ engine

def _engine_sigs(lib):
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    sig = {
        "df_engine_create": [vp, ctypes.c_size_t, vp, i32, ctypes.POINTER(vp)],
        "df_engine_job_bytes": [ctypes.POINTER(MeshDesc), ctypes.POINTER(ctypes.c_size_t)],
        "df_engine_admit": [vp, ctypes.POINTER(MeshDesc), dp, i32, ctypes.POINTER(i32)],
        "df_engine_step": [vp, i32],
        "df_engine_poll": [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)],
        "df_engine_active": [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)],
        "df_engine_force": [vp, i32, dp],
        "df_engine_get_field": [vp, i32, i32, i32, dp],
        "df_engine_release": [vp, i32],
        "df_engine_stats": [vp, ctypes.POINTER(ctypes.c_int64)],
        "df_engine_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        if f.argtypes is None:
            f.argtypes = args
            f.restype = ctypes.c_int


DF_EBUSY = -6


def engine_job_bytes(cfg: dict, precision=DF_FP64, tile_chunk=0) -> int:
    lib = _load()
    _engine_sigs(lib)
    d = _desc_of(cfg, precision, tile_chunk)
    n = ctypes.c_size_t()
    _ck(lib.df_engine_job_bytes(ctypes.byref(d), ctypes.byref(n)))
    return n.value


def _desc_of(cfg, precision, tile_chunk):
    return mesh_desc(cfg["nx"], cfg["ny"], cfg["nz"], cfg["nlevels"], cfg["dx0"], cfg.get("gamma", 5.0 / 3.0),
                     cfg.get("cfl", 0.4), precision, cfg.get("ghost_fine", 0), cfg.get("seed", 1),
                     cfg.get("noise_amp", 1e-6), tile_chunk, cfg.get("n1"), cfg.get("quadrant", False))


class Engine:
    """Continuous batching of independent runs (df_engine_*): one device arena
    (the HBM budget) allocated by PyTorch, the current stream as the replay
    stream."""

    def __init__(self, budget_bytes: int, *, nstreams=4, device="cuda"):
        import torch

        lib = _load()
        _engine_sigs(lib)
        self.device = torch.device(device)
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _ck(lib.df_engine_create(self.arena.data_ptr(), int(budget_bytes), self.stream.cuda_stream,
                                 int(nstreams), ctypes.byref(h)))
        self._h = h.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _ck(_load().df_engine_destroy(h))
            finally:
                self._h = None

    def admit(self, cfg: dict, nsteps: int, *, precision=DF_FP64, tile_chunk=0):
        """slot of the admitted job, or None when the budget or slots are exhausted"""
        d = _desc_of(cfg, precision, tile_chunk)
        pert = (ctypes.c_double * 5)(cfg["GM"], cfg["eps"], cfg["L"], cfg["mach"], cfg["chi"])
        slot = ctypes.c_int32()
        rc = _load().df_engine_admit(self._h, ctypes.byref(d), pert, int(nsteps), ctypes.byref(slot))
        if rc == DF_EBUSY:
            return None
        _ck(rc)
        return slot.value

    def step(self, n=1):
        _ck(_load().df_engine_step(self._h, int(n)))

    def poll(self, cap=1024):
        out = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        _ck(_load().df_engine_poll(self._h, out, cap, ctypes.byref(n)))
        return [out[i] for i in range(n.value)]

    def active(self):
        n = ctypes.c_int32()
        fb = ctypes.c_size_t()
        _ck(_load().df_engine_active(self._h, ctypes.byref(n), ctypes.byref(fb)))
        return n.value, fb.value

    def force(self, slot):
        out = np.zeros(4)
        _ck(_load().df_engine_force(self._h, int(slot), _dp(out)))
        return out

    def field(self, slot, level, name, shape):
        out = np.zeros(shape)
        _ck(_load().df_engine_get_field(self._h, int(slot), int(level), FIELDS[name], _dp(out)))
        return out

    def release(self, slot):
        _ck(_load().df_engine_release(self._h, int(slot)))

    def stats(self):
        out = (ctypes.c_int64 * 3)()
        _ck(_load().df_engine_stats(self._h, out))
        return {"replays": out[0], "captures": out[1], "batched": out[2]}
