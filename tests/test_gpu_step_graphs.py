"""df_step on nested runs replays HIP graphs of two coarse steps
(df_set_step_graphs): bitwise the same fields, force and force log as the
same run launched directly, over odd step counts (a direct last step), after a
change of the state (df_set_field), after a new perturber (a new capture), on
both hierarchies and the quadrant, in both precisions; replays interleaved
with unrelated GPU work and synchronisations."""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu

NAMES = ("rho", "e", "vx", "vy", "vz")


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


def _run(dfm, c, precision, graphs, quadrant=False):
    shape = (c["nx"], c["ny"] // 2, c["nz"] // 2) if quadrant else (c["nx"], c["ny"], c["nz"])
    n1 = c.get("n1")
    if n1 and quadrant:
        n1 = (n1[0], n1[1] // 2, n1[2] // 2)
    r = dfm.Run(*shape, nlevels=c["nlevels"], dx0=c["dx0"], gamma=c["gamma"], seed=c["seed"],
                noise_amp=c["noise_amp"], precision=precision, n1=n1, quadrant=quadrant)
    if quadrant:
        r.set_boundaries(1)
    r.set_step_graphs(graphs)
    r.set_perturber(c["GM"], c["eps"], c["L"], c["mach"], c["chi"])
    return r


def _same(a, b, nl):
    for lev in range(nl):
        for name in NAMES:
            assert np.array_equal(a.field(lev, name), b.field(lev, name)), (lev, name)
    assert np.array_equal(a.force(), b.force())
    la, lb = a.force_log(), b.force_log()
    assert la.shape == lb.shape and np.array_equal(la, lb)


CASES = [  # (ground cells, levels, finer-level cells, quadrant, precision)
    (32, 3, None, False, 0),
    (32, 3, None, False, 1),
    (64, 3, 32, False, 0),
    (32, 2, None, True, 0),
]


@pytest.mark.parametrize("n,nl,n1,quad,prec", CASES)
def test_graph_replays_equal_direct_launches(dfm, n, nl, n1, quad, prec):
    import torch

    _say(f"[graphs] {n}^3, {nl} levels, n1 {n1}, quadrant {quad}, precision {prec}")
    c = inputs.job(n, nl, 0.6, 2e-3, 0.1, 1e-3, seed=61, n1=n1)
    g = _run(dfm, c, prec, True, quad)
    d = _run(dfm, c, prec, False, quad)
    for steps in (5, 2, 3):
        g.step(steps)
        d.step(steps)
        x = torch.randn(1 << 18, device="cuda")
        _ = float((x * x).sum())
        torch.cuda.synchronize()
    _same(g, d, nl)
    # a changed state: the next replay starts from fresh signal speeds
    rho = g.field(nl - 1, "rho")
    rho[0, 0, 0] *= 1.001
    g.set_field(nl - 1, "rho", rho)
    d.set_field(nl - 1, "rho", rho)
    g.step(4)
    d.step(4)
    _same(g, d, nl)
    # a new perturber: the graphs are captured again
    g.set_perturber(c["GM"] * 2, c["eps"], c["L"], c["mach"], c["chi"])
    d.set_perturber(c["GM"] * 2, c["eps"], c["L"], c["mach"], c["chi"])
    g.step(6)
    d.step(6)
    _same(g, d, nl)
