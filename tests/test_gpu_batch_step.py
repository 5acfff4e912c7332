"""Batched stage and time-centred step through the C-ABI.

* rich_stage_batch over runs of uneven sizes, boundaries, parameters and
  Riemann solvers equals separate rich_stage calls bit for bit (the batch
  path uses a persistent grid and a different tile order than the single-run
  path, so this is also the tiling-independence check) and the oracle to
  1e-12; a failing run is reported alone and leaves the others untouched.
* rich_step follows the oracle's time-centred chain (identical start, same
  dt, meshes rebuilt by the host stage on each side), commits nothing on
  failure, and handles a static mesh.
"""
import numpy as np
import pytest

import oracle as O
import parity_util as U
from paper_1410_3219_amd import inputs as I
from paper_1410_3219_amd import tess as T

pytestmark = pytest.mark.gpu


def _runs():
    specs = [("sod", 17, 0, 0), ("wave", 23, 0, 0), ("sedov", 20, 1, 0), ("kh", 31, 0, 2),
             ("sod_angle", 9, 1, 1), ("gresho", 40, 0, 0), ("sod", 1, 0, 0)]
    out = []
    for name, k, riemann, limiter in specs:
        out.append(U.case(name, k=k, riemann=riemann, limiter=limiter, pass2=(k % 2 == 1)))
    return out


def _run_batch(cases, bad_run=None):
    import torch
    from paper_1410_3219_amd import rich as R
    meshes, srcs, bases, outs, hs, ps = [], [], [], [], [], []
    for r, (m, Qs, Qb, Xb, h, p) in enumerate(cases):
        if r == bad_run:
            Qb = Qb.copy()
            Qb[0, 0] = -1.0
        meshes.append(R.DeviceMesh.from_host(m))
        srcs.append(R.DeviceState.from_host(Qs, Xb))
        bases.append(R.DeviceState.from_host(Qb, Xb))
        o = R.DeviceState.empty_like(bases[-1])
        o.Q.fill_(float("nan"))
        outs.append(o)
        hs.append(h)
        ps.append(U.gpu_params(p))
    ws = R.batch_workspace([m.n_cells for m, *_ in cases])
    R.rich_stage_batch(meshes, srcs, bases, outs, hs, ps, ws)
    flags = R.rich_batch_flags(len(cases), ws)
    torch.cuda.synchronize()
    return [o.numpy() for o in outs], flags


def test_batch_equals_single_runs_bitwise_and_oracle():
    cases = _runs()
    res, flags = _run_batch(cases)
    assert flags == [0] * len(cases)
    for (m, Qs, Qb, Xb, h, p), (Qbat, Xbat) in zip(cases, res):
        Qg, Xg, f = U.gpu_stage(m, Qs, Qb, Xb, h, p)
        assert f == 0
        assert np.array_equal(Qbat, Qg) and np.array_equal(Xbat, Xg)
        U.check_stage(m, Qs, Qb, Xb, h, p, Qbat, Xbat, label="batched run")


def test_batch_with_acceleration_fields_equals_single_runs_and_oracle():
    """rich_stage_batch_accel over runs with and without a per-cell field
    (section 2.3 source term) equals separate rich_stage_accel / rich_stage
    calls bit for bit and the oracle's stage_accel / stage to 1e-12."""
    import torch
    from paper_1410_3219_amd import rich as R
    specs = [("sod", 17, 0, True), ("wave", 23, 1, True), ("sedov", 20, 0, False),
             ("kh", 31, 0, True), ("sod", 1, 1, True)]
    cases, fields = [], []
    for name, k, riemann, with_field in specs:
        c = U.case(name, k=k, riemann=riemann, pass2=(k % 2 == 1), g=(0.05, -0.3))
        m = c[0]
        rng = np.random.default_rng(k)
        a = np.stack([0.8 * np.sin(2 * np.pi * m.px) + rng.uniform(-0.1, 0.1, m.n_cells),
                      -0.5 * np.cos(2 * np.pi * m.py)]) if with_field else None
        cases.append(c)
        fields.append(a)
    meshes, srcs, bases, outs, hs, ps, accels = [], [], [], [], [], [], []
    for (m, Qs, Qb, Xb, h, p), a in zip(cases, fields):
        meshes.append(R.DeviceMesh.from_host(m))
        srcs.append(R.DeviceState.from_host(Qs, Xb))
        bases.append(R.DeviceState.from_host(Qb, Xb))
        o = R.DeviceState.empty_like(bases[-1])
        o.Q.fill_(float("nan"))
        outs.append(o)
        hs.append(h)
        ps.append(U.gpu_params(p))
        accels.append(None if a is None else torch.from_numpy(a).cuda())
    ws = R.batch_workspace([c[0].n_cells for c in cases])
    R.rich_stage_batch_accel(meshes, srcs, bases, outs, hs, ps, accels, ws)
    flags = R.rich_batch_flags(len(cases), ws)
    torch.cuda.synchronize()
    assert flags == [0] * len(cases)
    for r, ((m, Qs, Qb, Xb, h, p), a) in enumerate(zip(cases, fields)):
        Qbat, Xbat = outs[r].numpy()
        one = R.DeviceState.empty_like(bases[r])
        w1 = R.workspace(m.n_cells)
        if a is None:
            R.rich_stage(meshes[r], srcs[r], bases[r], one, h, ps[r], w1)
            ref = O.stage(m, Qs, Qb, Xb, h, p)
        else:
            R.rich_stage_accel(meshes[r], srcs[r], bases[r], one, h, ps[r], accels[r], w1)
            ref = O.stage_accel(m, Qs, Qb, Xb, h, p, a)
        torch.cuda.synchronize()
        Q1, X1 = one.numpy()
        assert np.array_equal(Qbat, Q1) and np.array_equal(Xbat, X1), r
        assert ref.status == 0
        U.check_stage(m, Qs, Qb, Xb, h, p, Qbat, Xbat, ref=ref, accel=a, label=f"batched run {r}")
    # a run with only one of its two components is rejected before any launch
    import ctypes as C
    n = len(cases)
    ax, ay = (C.c_void_p * n)(), (C.c_void_p * n)()
    ax[0] = accels[0].data_ptr()
    n_, mp, spp, bpp, opp, hh, ppp, _pc = R._batch_args(meshes, srcs, bases, outs, hs, ps)
    st = R.lib().rich_stage_batch_accel(n_, mp, spp, bpp, opp, hh, ppp, ax, ay,
                                        C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == R.RICH_E_INVAL


def test_batch_tile_shapes_bitwise_equal_and_autotune():
    """Every edge-tile shape (128, 256, 512 cells) gives the same results bit
    for bit; the autotuner times each and picks one of them."""
    import torch
    from paper_1410_3219_amd import rich as R
    cases = _runs()
    ref, _ = _run_batch(cases)
    meshes = [R.DeviceMesh.from_host(m) for m, *_ in cases]
    srcs = [R.DeviceState.from_host(Qs, Xb) for m, Qs, Qb, Xb, h, p in cases]
    bases = [R.DeviceState.from_host(Qb, Xb) for m, Qs, Qb, Xb, h, p in cases]
    hs = [c[4] for c in cases]
    ps = [U.gpu_params(c[5]) for c in cases]
    ws = R.batch_workspace([m.n_cells for m, *_ in cases])
    for tile in (128, 256, 512):
        outs = [R.DeviceState.empty_like(b) for b in bases]
        for o in outs:
            o.Q.fill_(float("nan"))
        plan = R.rich_stage_batch_prepare_tile(meshes, srcs, bases, outs, hs, ps, tile, ws)
        assert plan.flux_tile == tile
        R.rich_stage_batch_launch(plan, ws)
        assert R.rich_batch_flags(len(cases), ws) == [0] * len(cases)
        torch.cuda.synchronize()
        for (Qr, Xr), o in zip(ref, outs):
            Qo, Xo = o.numpy()
            assert np.array_equal(Qo, Qr) and np.array_equal(Xo, Xr), tile
    outs = [R.DeviceState.empty_like(b) for b in bases]
    best, ms = R.rich_stage_batch_autotune(meshes, srcs, bases, outs, hs, ps, ws, reps=2)
    assert best in (128, 256, 512) and all(v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())
    for (Qr, Xr), o in zip(ref, outs):
        assert np.array_equal(o.numpy()[0], Qr)
    with pytest.raises(R.RichError) as e:
        R.rich_stage_batch_prepare_tile(meshes, srcs, bases, outs, hs, ps, 64, ws)
    assert e.value.status == R.RICH_E_INVAL


def test_batch_failure_is_isolated():
    cases = _runs()
    good, _ = _run_batch(cases)
    res, flags = _run_batch(cases, bad_run=2)
    assert flags[2] != 0
    for r in range(len(cases)):
        if r == 2:
            continue
        assert flags[r] == 0
        assert np.array_equal(res[r][0], good[r][0])


def _oracle_chain(P, m, Q, X, dts, p):
    tf = lambda x, y, b, bc: T.rich_tess_build(x, y, b, bc)  # noqa: E731
    for dt in dts:
        Q, X, m, _, st = O.step(m, Q, X, dt, p, tf)
        assert st == 0
    return Q, X, m


def _gpu_chain(P, m, Q, X, dts, p, device_tess=False):
    import torch
    from paper_1410_3219_amd import rich as R
    ctx = R.RichCtx(device_tess=device_tess)
    ctx.set_mesh(m)
    s = R.DeviceState.from_host(Q, X)
    for dt in dts:
        ctx.step(s, dt, U.gpu_params(p))
    torch.cuda.synchronize()
    out = s.numpy()
    ctx.close()
    return out


def test_step_free_fall_and_gravity_chain():
    """rich_step under a uniform acceleration: the oracle's chain on a
    Kelvin-Helmholtz setup with gravity, and exact free fall of a uniform
    gas (the closed form the oracle is pinned to)."""
    P = I.kelvin_helmholtz(k=18)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    p = O.Params(gamma=P.gamma, gx=0.2, gy=-0.9)
    dt, _ = O.cfl_dt(m, Q, p)
    Qo, Xo, mo = _oracle_chain(P, m, Q, X, [dt] * 3, p)
    Qg, Xg = _gpu_chain(P, m, Q, X, [dt] * 3, p)
    eq, ex = U.errors(mo, Qg, Xg, Qo, Xo, Qo, p)
    assert (eq < 1e-11).all() and ex < 1e-12, (eq, ex)
    v0, g, gam = (0.3, -0.2), (0.7, -1.3), 5.0 / 3.0
    P = I.uniform_flow(k=16, v=v0, jitter=0.2, bc=1, gamma=gam)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X0 = np.stack([m.px, m.py])
    p = O.Params(gamma=gam, chi=0.0, gx=g[0], gy=g[1])
    Qg, Xg = _gpu_chain(P, m, Q, X0, [0.02] * 4, p)
    t = 0.08
    for q in range(2):
        assert np.max(np.abs(Qg[1 + q] / Qg[0] - (v0[q] + g[q] * t))) < 1e-13
        want = (X0[q] + v0[q] * t + 0.5 * g[q] * t * t) % 1.0
        assert np.max(np.abs((Xg[q] - want + 0.5) % 1.0 - 0.5)) < 1e-13


@pytest.mark.parametrize("name,motion", [("sod", 1), ("wave", 1), ("kh", 0)])
def test_step_extrapolated_fluxes_follows_oracle_chain(name, motion):
    if name == "sod":
        P = I.sod(k=24)
    elif name == "wave":
        P = I.advected_wave(k=20)
    else:
        P = I.kelvin_helmholtz(k=20)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    p = O.Params(gamma=P.gamma, motion=motion, integrator=1)
    dt, _ = O.cfl_dt(m, Q, p)
    Qo, Xo, mo = _oracle_chain(P, m, Q, X, [dt] * 4, p)
    Qg, Xg = _gpu_chain(P, m, Q, X, [dt] * 4, p)
    eq, ex = U.errors(mo, Qg, Xg, Qo, Xo, Qo, p)
    assert (eq < 1e-11).all() and ex < 1e-12, (eq, ex)


@pytest.mark.parametrize("name,motion", [("sod", 1), ("wave", 1), ("kh", 0)])
def test_step_follows_oracle_chain(name, motion):
    if name == "sod":
        P = I.sod(k=24)
    elif name == "wave":
        P = I.advected_wave(k=20)
    else:
        P = I.kelvin_helmholtz(k=20)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    p = O.Params(gamma=P.gamma, motion=motion)
    dt, _ = O.cfl_dt(m, Q, p)
    dts = [dt] * 4
    Qo, Xo, mo = _oracle_chain(P, m, Q, X, dts, p)
    Qg, Xg = _gpu_chain(P, m, Q, X, dts, p)
    eq, ex = U.errors(mo, Qg, Xg, Qo, Xo, Qo, p)
    print(f"\n{name} 4-step chain err {eq} x {ex}")
    assert (eq < 1e-11).all() and ex < 1e-12


def test_step_uncommitted_on_failure():
    from paper_1410_3219_amd import rich as R
    P = I.sod(k=12)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    Q[3, 7] = -1.0   # negative total energy in one cell
    X = np.stack([m.px, m.py])
    ctx = R.RichCtx()
    ctx.set_mesh(m)
    s = R.DeviceState.from_host(Q, X)
    with pytest.raises(R.RichError) as e:
        ctx.step(s, 0.01, R.Params())
    assert e.value.status in (R.RICH_E_DOMAIN, R.RICH_E_MESH)
    Qa, Xa = s.numpy()
    assert np.array_equal(Qa, Q) and np.array_equal(Xa, X)
    with pytest.raises(R.RichError):
        ctx.step(s, -1.0, R.Params())
    ctx.close()


def test_shock_tube_100_steps_drift_report():
    """Independent GPU and oracle chains over 100 steps of the 64^2 shock
    tube: a report, with a loose sanity bound (the two chains only share the
    initial state; round-off differences grow through the limiter)."""
    P = I.sod(k=64)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    p = O.Params(gamma=P.gamma)
    dts = []
    mm, QQ = m, Q
    dt, _ = O.cfl_dt(m, Q, p)
    dts = [dt] * 100
    Qo, Xo, mo = _oracle_chain(P, m, Q, X, dts, p)
    Qg, Xg = _gpu_chain(P, m, Q, X, dts, p)
    eq, ex = U.errors(mo, Qg, Xg, Qo, Xo, Qo, p)
    print(f"\nshock tube 64^2, 100 steps: drift per quantity {eq}, points {ex}")
    assert (eq < 1e-6).all()


def _step_batch_runs():
    """(problem, Params) of runs of uneven sizes: moving and static meshes,
    walls and periodic boxes, both Riemann solvers."""
    specs = [(I.sod(k=17, seed=3), dict(motion=1)),
             (I.advected_wave(k=23, seed=4), dict(motion=1)),
             (I.kelvin_helmholtz(k=14, seed=5), dict(motion=0)),
             (I.sod(k=9, seed=6, angle=0.4, gamma=1.4), dict(motion=1, riemann=1)),
             (I.gresho(k=20, seed=7), dict(motion=1, chi=0.5, eta=0.05)),
             (I.sod(k=15, seed=8), dict(motion=1, integrator=1)),
             (I.kelvin_helmholtz(k=12, seed=9), dict(motion=0, integrator=1))]
    out = []
    for P, kw in specs:
        m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
        X = np.stack([m.px, m.py])
        p = O.Params(gamma=P.gamma, **kw)
        dt, st = O.cfl_dt(m, Q, p)
        assert st == 0
        out.append((m, Q, X, p, dt))
    return out


def _batch_chain(runs, steps, bad_run=None, device_tess=lambda r: False, counts=None):
    import torch
    from paper_1410_3219_amd import rich as R
    ctxs, states = [], []
    for r, (m, Q, X, p, dt) in enumerate(runs):
        c = R.RichCtx(n_threads=1, device_tess=device_tess(r))
        c.set_mesh(m)
        Qr = Q.copy()
        if r == bad_run:
            Qr[3, 3] = -1.0
        ctxs.append(c)
        states.append(R.DeviceState.from_host(Qr, X))
    ws = R.batch_workspace([m.n_cells for m, *_ in runs])
    all_status = []
    for _ in range(steps):
        st = R.rich_step_batch(ctxs, states, [r[4] for r in runs],
                               [U.gpu_params(r[3]) for r in runs], ws, n_threads=4)
        all_status.append(st)
    torch.cuda.synchronize()
    out = [s.numpy() for s in states]
    meshes = [c.mesh().n_edges for c in ctxs]
    if counts is not None:
        counts.extend(c.tess_counts() for c in ctxs)
    for c in ctxs:
        c.close()
    return out, all_status, meshes


def test_step_batch_equals_separate_steps_bitwise():
    runs = _step_batch_runs()
    res, status, _ = _batch_chain(runs, 3)
    assert all(s == [0] * len(runs) for s in status), status
    for (m, Q, X, p, dt), (Qb, Xb) in zip(runs, res):
        Qs, Xs = _gpu_chain(None, m, Q, X, [dt] * 3, p)
        assert np.array_equal(Qb, Qs) and np.array_equal(Xb, Xs)


def test_step_batch_with_device_tess_equals_separate_steps_bitwise():
    """Half of the runs rebuild their meshes on the device: the batched step
    equals each run's own rich_step (with the same choice) bit for bit."""
    runs = _step_batch_runs()
    dev = lambda r: r % 2 == 0   # noqa: E731
    counts = []
    res, status, _ = _batch_chain(runs, 3, device_tess=dev, counts=counts)
    assert all(s == [0] * len(runs) for s in status), status
    for r, ((m, Q, X, p, dt), (Qb, Xb)) in enumerate(zip(runs, res)):
        Qs, Xs = _gpu_chain(None, m, Q, X, [dt] * 3, p, device_tess=dev(r))
        assert np.array_equal(Qb, Qs) and np.array_equal(Xb, Xs), r
        moving = p.motion == 1
        per_step = (1 if p.integrator == 1 else 2) if moving else 0
        assert counts[r] == ((3 * per_step, 0) if dev(r) else (0, 0)), (r, counts[r])


def test_step_batch_follows_oracle_chain():
    runs = _step_batch_runs()
    res, _, _ = _batch_chain(runs, 2)
    for (m, Q, X, p, dt), (Qb, Xb) in [(runs[r], res[r]) for r in (0, 1, 5)]:
        Qo, Xo, mo = _oracle_chain(None, m, Q, X, [dt] * 2, p)
        eq, ex = U.errors(mo, Qb, Xb, Qo, Xo, Qo, p)
        assert (eq < 1e-11).all() and ex < 1e-12, (eq, ex)


def test_step_batch_failure_is_isolated():
    from paper_1410_3219_amd import rich as R
    runs = _step_batch_runs()
    good, _, _ = _batch_chain(runs, 1)
    res, status, _ = _batch_chain(runs, 1, bad_run=1)
    assert status[0][1] == R.RICH_E_DOMAIN
    for r in range(len(runs)):
        if r == 1:
            # not committed: the state is the (bad) initial one
            Q = runs[1][1].copy()
            Q[3, 3] = -1.0
            assert np.array_equal(res[1][0], Q) and np.array_equal(res[1][1], runs[1][2])
            continue
        assert status[0][r] == 0
        assert np.array_equal(res[r][0], good[r][0]) and np.array_equal(res[r][1], good[r][1])


def test_batch_full_size_sampled_oracle_parity():
    """The batched workload at full size (256 shock-tube runs of 1k-65k
    cells, 4.0M cells in all, interface angle, gamma and rounding strength
    per run), in the configuration the benchmark replays: each stage as a
    prepared plan with its autotuned edge-tile shape.  Every run's flags are
    clear, and sampled runs (the smallest, the largest and six more) equal
    the oracle's stages to 1e-12 on the same inputs."""
    import torch
    from paper_1410_3219_amd import rich as R
    specs = I.batch_runs(256)
    runs = []
    for sp in specs:
        P = I.sod(k=sp["side"], seed=sp["seed"], angle=sp["angle"], gamma=sp["gamma"])
        hm = T.rich_tess_build(P.px, P.py, P.box, P.bc)
        Q0 = P.state(hm.area)
        X0 = np.stack([hm.px, hm.py])
        op = O.Params(gamma=sp["gamma"], chi=sp["chi"])
        dt, st = O.cfl_dt(hm, Q0, op)
        assert st == 0
        s0 = R.DeviceState.from_host(Q0, X0)
        runs.append(dict(hm=hm, Q0=Q0, X0=X0, op=op, dt=dt, dm=R.DeviceMesh.from_host(hm),
                         s0=s0, half=R.DeviceState.empty_like(s0),
                         out=R.DeviceState.empty_like(s0)))
    total = sum(r["hm"].n_cells for r in runs)
    assert 3.5e6 < total < 4.5e6
    ps = [U.gpu_params(r["op"]) for r in runs]
    ws = R.batch_workspace([r["hm"].n_cells for r in runs])
    a1 = ([r["dm"] for r in runs], [r["s0"] for r in runs], [r["s0"] for r in runs],
          [r["half"] for r in runs], [0.5 * r["dt"] for r in runs], ps)
    tile1, _ = R.rich_stage_batch_autotune(*a1, ws, reps=1)
    R.rich_stage_batch_launch(R.rich_stage_batch_prepare_tile(*a1, tile1, ws), ws)
    assert R.rich_batch_flags(len(runs), ws) == [0] * len(runs)
    for r in runs:   # the half-step meshes of the GPU's half-step points
        xh = r["half"].X.cpu().numpy()
        r["hmh"] = T.rich_tess_build(xh[0], xh[1], r["hm"].box, r["hm"].bc)
        r["dmh"] = R.DeviceMesh.from_host(r["hmh"])
    a2 = ([r["dmh"] for r in runs], [r["half"] for r in runs], [r["s0"] for r in runs],
          [r["out"] for r in runs], [r["dt"] for r in runs], ps)
    tile2, _ = R.rich_stage_batch_autotune(*a2, ws, reps=1)
    R.rich_stage_batch_launch(R.rich_stage_batch_prepare_tile(*a2, tile2, ws), ws)
    assert R.rich_batch_flags(len(runs), ws) == [0] * len(runs)
    torch.cuda.synchronize()
    sizes = np.array([r["hm"].n_cells for r in runs])
    pick = {int(sizes.argmin()), int(sizes.argmax())}
    pick |= set(np.random.default_rng(3).choice(len(runs), 6, replace=False).tolist())
    for k in sorted(pick):
        r = runs[k]
        Qh, Xh = r["half"].numpy()
        U.check_stage(r["hm"], r["Q0"], r["Q0"], r["X0"], 0.5 * r["dt"], r["op"], Qh, Xh,
                      label=f"run {k} stage 1")
        Qo, Xo = r["out"].numpy()
        U.check_stage(r["hmh"], Qh, r["Q0"], r["X0"], r["dt"], r["op"], Qo, Xo,
                      label=f"run {k} stage 2")
    print(f"\n{len(runs)} runs, {total} cells, tiles {tile1}/{tile2}, "
          f"{len(pick)} runs checked against the oracle")


@pytest.mark.parametrize("integrator", [0, 1])
def test_step_with_acceleration_field_follows_oracle_chain(integrator):
    """The step driver with a per-cell acceleration (rich_step_accel): three
    steps on a moving mesh of a Kelvin-Helmholtz setup follow the oracle's
    chain with the same field, both integrators."""
    import torch
    from paper_1410_3219_amd import rich as R
    P = I.kelvin_helmholtz(k=18, seed=7)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    p = O.Params(gamma=P.gamma, integrator=integrator, gx=0.05)
    a = np.stack([0.4 * np.sin(2 * np.pi * m.py), -0.6 * np.cos(2 * np.pi * m.px)])
    dts = [2e-3] * 3
    tf = lambda x, y, b, bc: T.rich_tess_build(x, y, b, bc)  # noqa: E731
    Qo, Xo, mo = Q, X, m
    for dt in dts:
        Qo, Xo, mo, _, st = O.step(mo, Qo, Xo, dt, p, tf, accel=a)
        assert st == 0
    ctx = R.RichCtx()
    ctx.set_mesh(m)
    s = R.DeviceState.from_host(Q, X)
    ag = torch.from_numpy(a).cuda()
    for dt in dts:
        ctx.step(s, dt, U.gpu_params(p), accel=ag)
    torch.cuda.synchronize()
    Qg, Xg = s.numpy()
    ctx.close()
    eq, ex = U.errors(mo, Qg, Xg, Qo, Xo, Q, p)
    print(f"\nintegrator {integrator}: 3 steps with a field, err {eq} x {ex}")
    assert (eq < 1e-11).all() and ex < 1e-11, (eq, ex)


def test_step_batch_with_acceleration_fields_equals_separate_steps_bitwise():
    """rich_step_batch_accel: runs with a per-cell field (moving and static
    meshes, both integrators) and runs without one equal separate
    rich_step_accel / rich_step calls bit for bit over three steps; a run
    with only one field component fails alone."""
    import torch
    from paper_1410_3219_amd import rich as R
    runs = _step_batch_runs()
    fields = []
    for r, (m, *_rest) in enumerate(runs):
        if r % 3 == 2:
            fields.append(None)
        else:
            fields.append(torch.from_numpy(np.stack(
                [0.4 * np.sin(2 * np.pi * m.py), -0.6 * np.cos(2 * np.pi * m.px)])).cuda())
    ctxs, states = [], []
    for m, Q, X, p, dt in runs:
        c = R.RichCtx(n_threads=1)
        c.set_mesh(m)
        ctxs.append(c)
        states.append(R.DeviceState.from_host(Q, X))
    ws = R.batch_workspace([m.n_cells for m, *_ in runs])
    for _ in range(3):
        st = R.rich_step_batch(ctxs, states, [r[4] for r in runs],
                               [U.gpu_params(r[3]) for r in runs], ws, n_threads=4,
                               accels=fields)
        assert st == [0] * len(runs), st
    torch.cuda.synchronize()
    for c in ctxs:
        c.close()
    for (m, Q, X, p, dt), a, s in zip(runs, fields, states):
        c = R.RichCtx(n_threads=1)
        c.set_mesh(m)
        one = R.DeviceState.from_host(Q, X)
        for _ in range(3):
            c.step(one, dt, U.gpu_params(p), accel=a)
        torch.cuda.synchronize()
        c.close()
        (Qb, Xb), (Q1, X1) = s.numpy(), one.numpy()
        assert np.array_equal(Qb, Q1) and np.array_equal(Xb, X1)
    # run 0 with ax only: that run fails with RICH_E_INVAL, the others commit
    import ctypes as C
    ctxs = []
    for m, Q, X, p, dt in runs[:2]:
        c = R.RichCtx(n_threads=1)
        c.set_mesh(m)
        ctxs.append(c)
    sts = [R.DeviceState.from_host(Q, X) for m, Q, X, p, dt in runs[:2]]
    ax, ay = (C.c_void_p * 2)(), (C.c_void_p * 2)()
    ax[0] = fields[0].data_ptr()
    ax[1], ay[1] = fields[1].data_ptr(), fields[1].data_ptr() + 8 * runs[1][0].n_cells
    cp = (C.c_void_p * 2)(*[c.h.value for c in ctxs])
    spp = (C.c_void_p * 2)(*[C.addressof(s.c()) for s in sts])
    dd = (C.c_double * 2)(*[r[4] for r in runs[:2]])
    pc = [U.gpu_params(r[3]).c() for r in runs[:2]]
    ppp = (C.c_void_p * 2)(*[C.addressof(x) for x in pc])
    users = (C.c_void_p * 2)(*[c.tess_user.value for c in ctxs])
    status = (C.c_int32 * 2)()
    ws2 = R.batch_workspace([r[0].n_cells for r in runs[:2]])
    rc = R.lib().rich_step_batch_accel(2, cp, spp, dd, ppp, ax, ay, ctxs[0].tess_fn,
                                       ctxs[0].release_fn, users, 1, status,
                                       C.c_void_p(ws2.data_ptr()), ws2.numel(), None)
    torch.cuda.synchronize()
    for c in ctxs:
        c.close()
    assert rc == R.RICH_E_INVAL and list(status) == [R.RICH_E_INVAL, R.RICH_OK]
