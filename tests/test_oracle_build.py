"""The oracle's optimisation flags change its speed, never its results: an
-O2 build and the -O3 / x86-64-v3 build the tests and the CPU baseline use give
bitwise-identical fields and forces (FMA contraction is off in both and
nothing reassociates).  CPU only."""
import numpy as np

from oracle import oracle
from oracle.oracle import Oracle


def test_o2_and_o3_builds_agree_bitwise(tmp_path):
    o2 = oracle.build(path=str(tmp_path / "liboracle_o2.so"), opt=("-O2",))
    kw = dict(nlevels=2, dx0=0.16, GM=0.01, eps=0.04, L=1e-3, mach=0.8, chi=0.1, noise_amp=1e-3, seed=5)
    a = Oracle(16, 16, 16, **kw)
    b = Oracle(16, 16, 16, lib_path=o2, **kw)
    a.step(4)
    b.step(4)
    for lev in range(2):
        for name in ("rho", "e", "vx", "vy", "vz"):
            assert np.array_equal(a.full_field(lev, name), b.full_field(lev, name)), (lev, name)
    assert np.array_equal(a.force(), b.force())
    assert np.array_equal(a.totals(), b.totals())
