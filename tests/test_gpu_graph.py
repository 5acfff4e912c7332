"""Prepared batched stages and HIP graphs.

rich_stage_batch_prepare + rich_stage_batch_launch equal rich_stage_batch
bit for bit; the launches of a time-centred batched step (both stages, the
half-step meshes built beforehand) captured once in a HIP graph give, on
every replay, exactly the eager step, with eager work and synchronisations
between the replays."""
import numpy as np
import pytest

import oracle as O
import parity_util as U
from paper_1410_3219_amd import inputs as I
from paper_1410_3219_amd import tess as T

pytestmark = pytest.mark.gpu


def _runs():
    """Uneven runs; moving meshes get their half-step mesh from the host
    stage on an oracle half stage (both sides see the same arrays)."""
    from paper_1410_3219_amd import rich as R
    out = []
    for P, kw in [(I.sod(k=19, seed=2), dict(motion=1)), (I.advected_wave(k=25, seed=3), {}),
                  (I.kelvin_helmholtz(k=16, seed=4), dict(motion=0)),
                  (I.sod(k=11, seed=5, angle=0.3), dict(motion=1, riemann=1))]:
        m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
        X = np.stack([m.px, m.py])
        p = O.Params(gamma=P.gamma, **kw)
        dt, _ = O.cfl_dt(m, Q, p)
        h1 = O.stage(m, Q, Q, X, 0.5 * dt, p)
        mh = T.rich_tess_build(h1.X[0], h1.X[1], P.box, P.bc) if p.motion else m
        cur = R.DeviceState.from_host(Q, X)
        out.append(dict(dm=R.DeviceMesh.from_host(m), dmh=R.DeviceMesh.from_host(mh), cur=cur,
                        half=R.DeviceState.empty_like(cur), nxt=R.DeviceState.empty_like(cur),
                        p=U.gpu_params(p), dt=dt, n=m.n_cells))
    return out


def _stage_args(runs, second):
    if not second:
        return ([r["dm"] for r in runs], [r["cur"] for r in runs], [r["cur"] for r in runs],
                [r["half"] for r in runs], [0.5 * r["dt"] for r in runs], [r["p"] for r in runs])
    return ([r["dmh"] for r in runs], [r["half"] for r in runs], [r["cur"] for r in runs],
            [r["nxt"] for r in runs], [r["dt"] for r in runs], [r["p"] for r in runs])


def test_prepare_launch_equals_batch_and_graph_replays():
    import torch
    from paper_1410_3219_amd import rich as R
    runs = _runs()
    ns = [r["n"] for r in runs]
    ws1, ws2 = R.batch_workspace(ns), R.batch_workspace(ns)
    # eager reference through rich_stage_batch
    R.rich_stage_batch(*_stage_args(runs, False), ws1)
    R.rich_stage_batch(*_stage_args(runs, True), ws2)
    torch.cuda.synchronize()
    ref = [(r["nxt"].Q.clone(), r["nxt"].X.clone()) for r in runs]
    assert R.rich_batch_flags(len(runs), ws1) == [0] * len(runs)
    assert R.rich_batch_flags(len(runs), ws2) == [0] * len(runs)

    # prepared plans, launched eagerly
    p1 = R.rich_stage_batch_prepare(*_stage_args(runs, False), ws1)
    p2 = R.rich_stage_batch_prepare(*_stage_args(runs, True), ws2)
    for r in runs:
        r["nxt"].Q.fill_(float("nan"))
    R.rich_stage_batch_launch(p1, ws1)
    R.rich_stage_batch_launch(p2, ws2)
    torch.cuda.synchronize()
    for r, (q, x) in zip(runs, ref):
        assert torch.equal(r["nxt"].Q, q) and torch.equal(r["nxt"].X, x)

    # the same two launches captured once and replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        R.rich_stage_batch_launch(p1, ws1, s)
        R.rich_stage_batch_launch(p2, ws2, s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        R.rich_stage_batch_launch(p1, ws1, s)
        R.rich_stage_batch_launch(p2, ws2, s)
    torch.cuda.synchronize()
    for rep in range(3):
        for r in runs:                      # eager work between the replays
            r["nxt"].Q.fill_(float("nan"))
            r["half"].X.mul_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for r, (q, x) in zip(runs, ref):
            assert torch.equal(r["nxt"].Q, q) and torch.equal(r["nxt"].X, x), rep
        assert R.rich_batch_flags(len(runs), ws2) == [0] * len(runs)
    del g


def test_launch_rejects_bad_plans():
    from paper_1410_3219_amd import rich as R
    ws = R.batch_workspace([100])
    bad = R.RichBatchPlan()
    with pytest.raises(R.RichError):
        R.rich_stage_batch_launch(bad, ws)
