"""The allocation-free force entry point (df_force_density, partials in the
library's own device array) against the run-based df_force it mirrors: two
calls in a row on one GPU, the second over a smaller field, each within the
force bar of the parity tests (1e-9 of the force's norm)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(dfm, n, steps, seed):
    nx, ny, nz = n
    g = dfm.Run(nx, ny, nz, dx0=0.05, seed=seed, noise_amp=1e-3)
    g.set_perturber(0.01, 0.05, 2e-3, 0.8, 0.1)
    g.step(steps)
    return g


def test_force_density_matches_df_force_twice():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_03191_amd as dfm

    outs = []
    for n, steps, seed in (((48, 40, 32), 12, 3), ((16, 12, 8), 5, 4)):
        print(f"[no-alloc] n={n} steps={steps}", flush=True)
        g = _run(dfm, n, steps, seed)
        want = g.force()[:3]
        rho = torch.from_numpy(np.ascontiguousarray(g.field(0, "rho"))).to("cuda")
        out = dfm.force_density(rho, 0.05, 0.01, 0.05, 1.0)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-9 * np.linalg.norm(want), (n, got, want)
        outs.append((out, got))
    # the first call's output is the caller's and stays as written
    assert np.array_equal(outs[0][0].cpu().numpy(), outs[0][1])
