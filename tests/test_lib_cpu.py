"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point that include/df.h declares, and validates descriptions."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "df.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(df_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("df_init_mesh", "df_set_perturber", "df_step", "df_force"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1812_03191_amd as dfm

    lib = ctypes.CDLL(dfm.lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("bad", [
    dict(nx=33), dict(nlevels=0), dict(nlevels=13), dict(dx0=0.0), dict(gamma=1.0),
    dict(cfl=0.0), dict(cfl=1.5), dict(precision=7), dict(nlevels=2, nx=18),
    dict(nlevels=2, nx=12, ny=12, nz=12), dict(nlevels=2, ghost_fine=6), dict(noise_amp=0.7),
    dict(quadrant=2),
])
def test_init_mesh_rejects_bad_descriptions(bad):
    import paper_1812_03191_amd as dfm

    kw = dict(nx=16, ny=16, nz=16, nlevels=1, dx0=0.1)
    kw.update(bad)
    with pytest.raises(dfm.DFError) as ei:
        dfm.init_mesh(**kw)
    assert ei.value.code == -1


def test_required_bytes_scales_with_mesh():
    import paper_1812_03191_amd as dfm

    a = dfm.init_mesh(32, 32, 32, 1, 0.1)
    b = dfm.init_mesh(64, 64, 64, 1, 0.1)
    c = dfm.init_mesh(64, 64, 64, 3, 0.1)
    na, nb, nc = (dfm.required_bytes(h) for h in (a, b, c))
    # level 0 stores cells and faces 0..n (no ghosts), rows padded to 16 doubles
    assert 8 * 20 * 33 ** 3 <= na < 2 * 8 * 20 * 33 ** 3
    assert nb > 6 * na
    assert nc > 3 * nb
    for h in (a, b, c):
        dfm.destroy(h)


def test_calls_out_of_order_fail_cleanly():
    import paper_1812_03191_amd as dfm

    h = dfm.init_mesh(16, 16, 16, 1, 0.1)
    with pytest.raises(dfm.DFError) as ei:
        dfm.step(h, 1)
    assert ei.value.code == -2
    with pytest.raises(dfm.DFError):
        dfm.set_perturber(h, 0.01, 0.0, 0.0, 0.5, 0.1)
    dfm.destroy(h)


def test_engine_job_bytes_on_host():
    import paper_1812_03191_amd as dfm

    cfg = dict(nx=48, ny=48, nz=48, nlevels=1, dx0=0.1)
    b64 = dfm.engine_job_bytes(cfg, dfm.DF_FP64)
    b32 = dfm.engine_job_bytes(cfg, dfm.DF_FP32)
    assert b64 % 256 == 0 and b32 % 256 == 0
    assert 0.45 < b32 / b64 < 0.6


def test_serving_work_count():
    from paper_1812_03191_amd.serve import job_cell_updates

    assert job_cell_updates(dict(nx=32, ny=32, nz=32, nlevels=3), 10) == 10 * 32 ** 3 * 7


def test_launch_switches_need_a_bound_run():
    # before df_bind the fusion switches report an out-of-order call; a null
    # handle is a bad argument (their values are checked on the GPU)
    import paper_1812_03191_amd as dfm
    from paper_1812_03191_amd import _lib

    h = dfm.init_mesh(16, 16, 16, 1, 0.1)
    lib = _lib._load()
    for fn in (lib.df_set_kick_fusion, lib.df_set_transport_fusion, lib.df_set_finish_fusion,
               lib.df_set_step_graphs):
        assert fn(h, 1) == -2
        assert fn(None, 1) == -1
    dfm.destroy(h)


def test_force_density_validates_before_any_device_call():
    # argument checks come first: no GPU is touched for a rejected call
    import paper_1812_03191_amd as dfm
    from paper_1812_03191_amd import _lib

    lib = _lib._load()
    out = ctypes.c_void_p(16)  # never dereferenced: every call below is rejected
    rho = ctypes.c_void_p(16)
    assert lib.df_force_density(None, 8, 8, 8, 0.1, 0.01, 0.0, 1.0, out, None) == -1
    assert lib.df_force_density(rho, 8, 8, 8, 0.1, 0.01, 0.0, 1.0, None, None) == -1
    assert lib.df_force_density(rho, 7, 8, 8, 0.1, 0.01, 0.0, 1.0, out, None) == -1
    assert lib.df_force_density(rho, 8, 8, 0, 0.1, 0.01, 0.0, 1.0, out, None) == -1
    assert lib.df_force_density(rho, 8, 8, 8, 0.0, 0.01, 0.0, 1.0, out, None) == -1
    assert lib.df_force_density(rho, 8, 8, 8, 0.1, -1.0, 0.0, 1.0, out, None) == -1
    assert lib.df_force_density(rho, 8, 8, 8, 0.1, 0.01, float("nan"), 1.0, out, None) == -1
    big = 2048  # 2^33 cells: above the stated maximum
    assert lib.df_force_density(rho, big, big, big, 0.1, 0.01, 0.0, 1.0, out, None) == -1
    assert "MAX_CELLS" in lib.df_last_error().decode()
    assert dfm.DFError


def test_bench_refuses_more_than_one_gpu():
    # the measurement runs on one GPU: asking for more exits with a message
    # before any device work
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2, (r.returncode, r.stderr)
    assert "one GPU" in r.stderr and not r.stdout.strip()
