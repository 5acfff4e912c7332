"""Cell-rounding parameter sweep (section 6) through the batched step: each
run of the sweep follows the oracle's own time-centred chain with the same
(chi, eta), and the density error L of eq. (Lgresho) agrees."""
import numpy as np
import pytest

import oracle as O
import parity_util as U
from paper_1410_3219_amd import tess as T

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("device_tess", [False, True])
def test_sweep_runs_follow_oracle_chains(device_tess):
    from paper_1410_3219_amd import sweep as SW
    grid = [(0.01, 0.001), (0.15, 0.02), (1.0, 0.5), (0.5, 0.005)]
    sw = SW.Sweep(grid, k=16, n_threads=4, device_tess=device_tess)
    P, m = sw.problem, sw.mesh0
    # per-run dt from the oracle's Courant step, fixed for the 3 steps
    dts = []
    for chi, eta in grid:
        p = O.Params(gamma=P.gamma, chi=chi, eta=eta, motion=1)
        dt, st = O.cfl_dt(m, sw.Q0, p)
        assert st == 0
        dts.append(dt)
    for _ in range(3):
        st = sw.step(dts=dts)
        assert st == [0] * len(grid)
    L_gpu = sw.density_L()
    tf = lambda x, y, b, bc: T.rich_tess_build(x, y, b, bc)  # noqa: E731
    for r, (chi, eta) in enumerate(grid):
        p = O.Params(gamma=P.gamma, chi=chi, eta=eta, motion=1)
        Q, X, mm = sw.Q0, sw.X0, m
        for _ in range(3):
            Q, X, mm, _, st = O.step(mm, Q, X, dts[r], p, tf)
            assert st == 0
        Qg, Xg = sw.states[r].numpy()
        eq, ex = U.errors(mm, Qg, Xg, Q, X, Q, p)
        assert (eq < 1e-11).all() and ex < 1e-12, (r, eq, ex)
        L_o = float(np.mean(np.abs(Q[0] / mm.area - 1.0)))
        assert abs(L_gpu[r] - L_o) <= 1e-9 * max(L_o, 1e-12) + 1e-15, (r, L_gpu[r], L_o)
    # different rounding strengths move the points differently
    assert len({round(x, 15) for x in L_gpu}) > 1
    assert sw.tess_counts() == ((2 * 3 * len(grid), 0) if device_tess else (0, 0))
    sw.close()


def test_sweep_courant_steps_reach_end_time():
    from paper_1410_3219_amd import sweep as SW
    sw = SW.Sweep(SW.chi_eta_grid(2, 2), k=12, n_threads=4)
    sw.run(t_end=0.02)
    assert all(s == 0 for s in sw.status)
    assert np.allclose(sw.t, 0.02, rtol=0, atol=1e-15)
    L = sw.density_L()
    assert all(np.isfinite(L)) and max(L) < 0.05
    sw.close()
