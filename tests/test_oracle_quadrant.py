"""The paper's quadrant (Sect. 3.4): the domain y > 0, z > 0 bounded by the
perturber's mirror planes (here the flow is along x, the paper's along z),
with every nested level anchored at the planes.  Pinned by the full box,
which holds the quadrant's mirror images: a quadrant run equals the quarter
y, z > 0 of the full box run bitwise, field by field and level by level, on
one level, on the central-half hierarchy and on the quarter hierarchy of
Sects. 4.1.3 and 4.2.2; its force (the whole gas's, mirror images included)
and totals agree with the full box's to rounding.  CPU only."""
import numpy as np
import pytest

from oracle.oracle import Oracle

NAMES = ("rho", "e", "vx", "vy", "vz")


def _runs(n, nl, n1, steps, **kw):
    base = dict(nlevels=nl, gamma=1.4, noise_amp=0.0, GM=5e-3, eps=0.0, L=2e-3, mach=0.4, chi=0.1, bcmode=1)
    base.update(kw)
    full = Oracle(n, n, n, n1=(n1, n1, n1) if n1 else None, **base)
    quad = Oracle(n, n // 2, n // 2, n1=(n1, n1 // 2, n1 // 2) if n1 else None, quadrant=True, **base)
    full.step(steps)
    quad.step(steps)
    return full, quad


CASES = [(32, 1, None, 12, 0.05), (32, 2, None, 4, 0.16), (64, 3, 32, 3, 0.16), (32, 4, None, 2, 0.32)]


@pytest.mark.parametrize("n,nl,n1,steps,dx0", CASES)
def test_quadrant_is_a_quarter_of_the_full_box(n, nl, n1, steps, dx0):
    full, quad = _runs(n, nl, n1, steps, dx0=dx0)
    assert quad.time == full.time
    for lev in range(nl):
        m = n if lev == 0 or not n1 else n1
        h = m // 2
        for name in NAMES:
            a = full.full_field(lev, name)
            b = quad.full_field(lev, name)
            sub = a[h:, h:, :]
            assert sub.shape == b.shape, (lev, name, sub.shape, b.shape)
            assert np.array_equal(sub, b), (lev, name, float(np.max(np.abs(sub - b))))
    Ff, Fq = full.force(), quad.force()
    assert Fq[1] == 0.0 and Fq[2] == 0.0
    assert abs(Fq[0] - Ff[0]) <= 1e-13 * abs(Ff[0]), (Fq, Ff)
    tf, tq = full.totals(), quad.totals()
    assert np.max(np.abs(tq[:3] - tf[:3]) / np.abs(tf[:3])) < 1e-13, (tq, tf)


def test_quadrant_needs_the_boundary_list():
    with pytest.raises(ValueError):
        Oracle(32, 16, 16, dx0=0.05, quadrant=True, bcmode=0)


def test_quadrant_heat_release_is_a_quarter():
    # the 8 cells around the perturber's vertex: 2 of them in the quadrant,
    # each with 1/8 of L dt (the other 6 are its mirror images)
    o = Oracle(16, 8, 8, dx0=0.1, quadrant=True, bcmode=1, eps=0.0)
    w = o.heat_weights(0)
    assert np.count_nonzero(w) == 2
    assert np.all(w[w > 0] == 0.125)
    assert w[0, 0, 7] == 0.125 and w[0, 0, 8] == 0.125
