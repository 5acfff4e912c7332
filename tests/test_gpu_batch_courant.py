"""Batched stages whose steps are taken on the device
(rich_stage_batch_prepare_courant, section 2.3 Courant condition), through
the C-ABI: every run's step and both stages of its time-centred step equal
the single-run device-step path (rich_stage_courant, rich_stage_dt_of) bit
for bit, the steps agree with the oracle's Courant condition, the first
stage agrees with the oracle's stage, and the whole step replays from one
captured graph with identical results."""
import numpy as np
import pytest

import oracle as O
import parity_util as U

pytestmark = pytest.mark.gpu

# uneven sizes, walls and periodic boxes, both Riemann solvers (two flux
# groups), static and moving meshes; the last run is one cell
SPECS = [("sod", 17, 0, 1), ("wave", 23, 0, 1), ("sedov", 20, 1, 1), ("kh", 31, 0, 0),
         ("sod_angle", 9, 1, 1), ("gresho", 40, 0, 1), ("sod", 1, 0, 1)]


def _runs():
    from paper_1410_3219_amd import rich as R
    runs = []
    for name, k, riemann, motion in SPECS:
        m, Q, _, X, _, p = U.case(name, k=k, riemann=riemann, motion=motion)
        runs.append(dict(m=m, Q=Q, X=X, p=p, gp=U.gpu_params(p), dm=R.DeviceMesh.from_host(m),
                         s=R.DeviceState.from_host(Q, X)))
    return runs


def _alone(run):
    """Both stages of one run through the single-run device-step path."""
    import torch
    from paper_1410_3219_amd import rich as R
    n = run["m"].n_cells
    ws = R.workspace(n)
    half = R.DeviceState.empty_like(run["s"])
    R.rich_stage_courant(run["dm"], run["s"], run["s"], half, 0.5, run["gp"], ws)
    assert R.rich_stage_flags(ws) == 0
    dt = R.rich_stage_dt(ws)
    Qh, Xh = half.numpy()
    m = run["m"]
    mh = U.host_mesh(Xh[0], Xh[1], m.box, m.bc) if run["p"].motion else m
    dmh = R.DeviceMesh.from_host(mh)
    out = R.DeviceState.empty_like(run["s"])
    ws2 = R.workspace(n)
    R.rich_stage_dt_of(dmh, half, run["s"], out, 1.0, ws, run["gp"], ws2)
    assert R.rich_stage_flags(ws2) == 0
    torch.cuda.synchronize()
    return dict(dt=dt, Qh=Qh, Xh=Xh, out=out.numpy(), dmh=dmh)


def _prepare1(R, runs, halves, ws1):
    n = len(runs)
    return R.rich_stage_batch_prepare_courant([r["dm"] for r in runs], [r["s"] for r in runs],
                                              [r["s"] for r in runs], halves, [0.5] * n,
                                              [r["gp"] for r in runs], ws1)


def _prepare2(R, runs, alone, halves, outs, ws1, ws2):
    n = len(runs)
    return R.rich_stage_batch_prepare_courant([a["dmh"] for a in alone], halves,
                                              [r["s"] for r in runs], outs, [1.0] * n,
                                              [r["gp"] for r in runs], ws2, dt_ws=ws1)


@pytest.mark.parametrize("same_ws", [False, True])
def test_batch_courant_step_equals_single_runs_bitwise(same_ws):
    import torch
    from paper_1410_3219_amd import rich as R
    runs = _runs()
    alone = [_alone(r) for r in runs]
    n = len(runs)
    ws1 = R.batch_workspace([r["m"].n_cells for r in runs])
    ws2 = ws1 if same_ws else R.batch_workspace([r["m"].n_cells for r in runs])
    halves = [R.DeviceState.empty_like(r["s"]) for r in runs]
    outs = [R.DeviceState.empty_like(r["s"]) for r in runs]
    for s in halves + outs:
        s.Q.fill_(float("nan"))
        s.X.fill_(float("nan"))
    # with one workspace the second prepare replaces the first stage's
    # descriptors, so each stage is prepared right before its launch
    p1 = _prepare1(R, runs, halves, ws1)
    assert p1.courant == 1
    R.rich_stage_batch_launch(p1, ws1)
    assert R.rich_batch_flags(n, ws1) == [0] * n
    dts = R.rich_batch_dt(n, ws1)
    p2 = _prepare2(R, runs, alone, halves, outs, ws1, ws2)
    assert p2.courant == 0
    if same_ws:   # the first plan is no longer the workspace's: rejected on the host
        with pytest.raises(R.RichError) as e:
            R.rich_stage_batch_launch(p1, ws1)
        assert e.value.status == R.RICH_E_INVAL
    R.rich_stage_batch_launch(p2, ws2)
    assert R.rich_batch_flags(n, ws2) == [0] * n
    assert R.rich_batch_dt(n, ws1) == dts          # the second stage left the steps alone
    torch.cuda.synchronize()
    for r, a, dt, h, o in zip(runs, alone, dts, halves, outs):
        dt_ref, st = O.cfl_dt(r["m"], r["Q"], r["p"])
        assert st == 0
        assert dt == a["dt"], (dt, a["dt"])
        assert abs(dt - dt_ref) <= 1e-13 * dt_ref, (dt, dt_ref)
        Qh, Xh = h.numpy()
        assert np.array_equal(Qh, a["Qh"]) and np.array_equal(Xh, a["Xh"])
        Qo, Xo = o.numpy()
        assert np.array_equal(Qo, a["out"][0]) and np.array_equal(Xo, a["out"][1])
        U.check_stage(r["m"], r["Q"], r["Q"], r["X"], 0.5 * dt, r["p"], Qh, Xh,
                      label="batched Courant stage 1")


def test_batch_courant_step_replays_from_one_graph():
    """Both prepared stages captured once; each replay (with eager work and
    synchronisations between replays) reproduces the eager step bit for bit."""
    import torch
    from paper_1410_3219_amd import rich as R
    runs = _runs()
    alone = [_alone(r) for r in runs]
    n = len(runs)
    ws1 = R.batch_workspace([r["m"].n_cells for r in runs])
    ws2 = R.batch_workspace([r["m"].n_cells for r in runs])
    halves = [R.DeviceState.empty_like(r["s"]) for r in runs]
    outs = [R.DeviceState.empty_like(r["s"]) for r in runs]
    p1 = _prepare1(R, runs, halves, ws1)
    p2 = _prepare2(R, runs, alone, halves, outs, ws1, ws2)
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):      # warm-up on the capture stream
        R.rich_stage_batch_launch(p1, ws1, gs)
        R.rich_stage_batch_launch(p2, ws2, gs)
    torch.cuda.current_stream().wait_stream(gs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        R.rich_stage_batch_launch(p1, ws1, gs)
        R.rich_stage_batch_launch(p2, ws2, gs)
    torch.cuda.synchronize()
    for rep in range(3):
        for s in halves + outs:
            s.Q.fill_(float("nan"))
            s.X.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert R.rich_batch_flags(n, ws1) == [0] * n and R.rich_batch_flags(n, ws2) == [0] * n
        dts = R.rich_batch_dt(n, ws1)
        for a, dt, h, o in zip(alone, dts, halves, outs):
            assert dt == a["dt"]
            Qh, Xh = h.numpy()
            assert np.array_equal(Qh, a["Qh"]) and np.array_equal(Xh, a["Xh"]), rep
            Qo, Xo = o.numpy()
            assert np.array_equal(Qo, a["out"][0]) and np.array_equal(Xo, a["out"][1]), rep
    del graph
