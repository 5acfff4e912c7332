"""Serving loop (continuous batching of step requests): a session served
among many others ends in exactly the state of the same steps run alone with
single-run stage calls and within the parity bars of the oracle's chain of
the same steps, launches do carry sessions of different templates, every
request completes, and admission keeps the device memory of admitted
sessions within the budget."""
import numpy as np
import pytest

import oracle as O
import parity_util as U

pytestmark = pytest.mark.gpu


def _alone(tpl, steps):
    import torch
    from paper_1410_3219_amd import rich as R
    cur = R.DeviceState.from_host(tpl.Q0, tpl.X0)
    half = R.DeviceState.empty_like(cur)
    nxt = R.DeviceState.empty_like(cur)
    ws = R.workspace(tpl.n)
    for _ in range(steps):
        R.rich_stage(tpl.mesh, cur, cur, half, 0.5 * tpl.dt, tpl.params, ws)
        R.rich_stage(tpl.mesh, half, cur, nxt, tpl.dt, tpl.params, ws)
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    return cur.numpy()


def test_served_sessions_match_alone_bitwise():
    from paper_1410_3219_amd import serve as S
    tpl = S.build_templates([400, 2500, 9000, 1200], ["sod", "sedov", "sod", "sedov"])
    budget = 3 * S.Server.session_bytes(9000)
    res, srv = S.run(tpl, rate=3000.0, duration=0.05, steps_per_session=3,
                     hbm_budget_bytes=budget, keep_final=True)
    assert res["requests"] == len(S.I.poisson_arrivals(3000.0, 0.05, 9))
    assert 0 < srv.max_used <= budget
    print(f"\nserved: {res['launches']} launches, max batch {res['max_batch']}, "
          f"{res['mixed_launches']} with sessions of different templates", flush=True)
    assert res["max_batch"] >= 2 and res["mixed_launches"] >= 1
    # every session's final state equals its steps run alone
    per_sess = {}
    for r in srv.done:
        per_sess[r.sid] = per_sess.get(r.sid, 0) + 1
    assert all(not s.admitted for s in srv.sessions.values())
    checked = 0
    for sid, sess in srv.sessions.items():
        ref = _alone(sess.tpl, per_sess[sid])
        assert sess.final is not None
        assert np.array_equal(sess.final[0], ref[0]) and np.array_equal(sess.final[1], ref[1])
        checked += 1
    assert checked == len(srv.sessions)


def _oracle_chain_static(tpl, steps):
    """The oracle's time-centred steps of a static-mesh template: stage 1
    (dt/2) and stage 2 (dt) on the template's own mesh, rebuilt on the host
    from its points; returns (mesh, final Q, last stage's diagnostics and
    inputs for the per-cell bar)."""
    from paper_1410_3219_amd import tess as T
    m = T.rich_tess_build(tpl.X0[0], tpl.X0[1], tpl.mesh.box, tpl.mesh.bc)
    assert np.array_equal(m.area, np.asarray(R_area(tpl)))
    p = O.Params(gamma=tpl.params.gamma, motion=0)
    Q, X = tpl.Q0.copy(), tpl.X0.copy()
    last = None
    for _ in range(steps):
        s1 = O.stage(m, Q, Q, X, 0.5 * tpl.dt, p)
        assert s1.status == 0
        s2 = O.stage(m, s1.Q, Q, X, tpl.dt, p, diag=True)
        assert s2.status == 0
        last = (s1.Q, Q, X, s2)
        Q, X = s2.Q, s2.X
    return m, Q, X, p, last


def R_area(tpl):
    from paper_1410_3219_amd import rich as R
    return R.mesh_to_host(tpl.mesh).area


def test_mixed_launch_sessions_follow_oracle_chains():
    """Sessions of four templates (shock tubes and point explosions of
    different sizes) with all their requests queued at once: the first
    launch carries all four, so their stages run in one batched launch.
    Each session ends bit for bit as its steps run alone, and within the
    parity bars of the oracle's chain of the same steps (per conserved
    quantity, and per cell against the last stage's terms)."""
    import time
    from paper_1410_3219_amd import serve as S
    tpl = S.build_templates([900, 1600, 2500, 1200], ["sod", "sedov", "sod", "sedov"])
    srv = S.Server(tpl, hbm_budget_bytes=1 << 30, keep_final=True)
    steps = 3
    for sid in range(4):
        srv.open_session(sid, sid, steps)
    rid = 0
    for _ in range(steps):
        for sid in range(4):
            srv.submit(rid, sid, 0.0)
            rid += 1
    t0 = time.perf_counter()
    srv.drain(lambda: time.perf_counter() - t0, timeout_s=120.0)
    assert len(srv.done) == 4 * steps and not srv.failed
    assert srv.launch_templates[0] == (0, 1, 2, 3), srv.launch_templates
    for sid in range(4):
        sess = srv.sessions[sid]
        ref = _alone(sess.tpl, steps)
        assert np.array_equal(sess.final[0], ref[0]) and np.array_equal(sess.final[1], ref[1])
        m, Qo, Xo, p, (Qs, Qb, Xb, diag) = _oracle_chain_static(sess.tpl, steps)
        eq, ex = U.errors(m, sess.final[0], sess.final[1], Qo, Xo, Qo, p)
        ec, where = U.cell_errors(m, sess.final[0], Qb, Qo, sess.tpl.dt, p, diag, Qs=Qs)
        print(f"\nserved {sess.tpl.name}: {steps} steps vs oracle chain: per quantity {eq}, "
              f"per cell {ec}", flush=True)
        assert (eq < 1e-11).all() and ex < 1e-12, (sess.tpl.name, eq, ex)
        assert (ec < 1e-11).all(), (sess.tpl.name, ec, where)


def test_flagged_session_is_evicted_and_others_go_on():
    """A session whose state turns invalid is evicted at its first flagged
    step (its memory released, its requests failed, later ones rejected)
    while the sessions batched with it finish bit for bit as alone."""
    import time
    from paper_1410_3219_amd import serve as S
    tpl = S.build_templates([400, 900], ["sod", "sedov"])
    srv = S.Server(tpl, hbm_budget_bytes=1 << 30, keep_final=True)
    steps = 3
    for sid in range(3):
        srv.open_session(sid, sid % 2, steps)
    srv._admit()
    assert all(s.admitted for s in srv.sessions.values())
    srv.sessions[1].cur.Q[0, 5] = -1.0          # negative mass in one cell of session 1
    rid = 0
    for _ in range(steps):
        for sid in range(3):
            srv.submit(rid, sid, 0.0)
            rid += 1
    t0 = time.perf_counter()
    srv.drain(lambda: time.perf_counter() - t0, timeout_s=120.0)
    bad = srv.sessions[1]
    assert bad.error != 0 and not bad.admitted
    assert sorted(r.rid for r in srv.failed) == [1, 4, 7]
    assert srv.used == 0
    # the evicted session's final state is its state before the failed step
    assert bad.final[0][0, 5] == -1.0
    srv.submit(rid, 1, 1.0)                      # a late request of the evicted session
    assert srv.failed[-1].rid == rid and not srv.queue
    for sid in (0, 2):
        s = srv.sessions[sid]
        assert s.error == 0
        ref = _alone(s.tpl, steps)
        assert np.array_equal(s.final[0], ref[0]) and np.array_equal(s.final[1], ref[1])


def _alone_moving(tpl, steps):
    """The same steps with single-run stages and re-tessellations."""
    import torch
    from paper_1410_3219_amd import rich as R
    m = tpl.mesh
    cur = R.DeviceState.from_host(tpl.Q0, tpl.X0)
    half = R.DeviceState.empty_like(cur)
    nxt = R.DeviceState.empty_like(cur)
    ws = R.workspace(tpl.n)
    bufs = [R.DeviceMeshBufs(m.n_cells, m.box, m.bc) for _ in range(3)]
    rws = R.retess_workspace(tpl.n)
    mesh, b = m, 0
    for _ in range(steps):
        hb, nb = bufs[b % 3], bufs[(b + 1) % 3]
        R.rich_stage(mesh, cur, cur, half, 0.5 * tpl.dt, tpl.params, ws)
        R.rich_retess(mesh, half.X, hb, rws)
        assert R.rich_retess_result(rws)[0] == 0
        R.rich_stage(hb.mesh(), half, cur, nxt, tpl.dt, tpl.params, ws)
        R.rich_retess(hb.mesh(), nxt.X, nb, rws)
        assert R.rich_retess_result(rws)[0] == 0
        mesh, b = nb.mesh(), b + 2
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    return cur.numpy()


def test_served_moving_sessions_match_alone_bitwise():
    """Sessions on moving meshes (each step: stage 1, device re-tessellation
    of the half-step points, stage 2, re-tessellation of the new points, all
    batched over the launch's sessions) end in exactly the state of the same
    steps run alone; the points do move."""
    from paper_1410_3219_amd import serve as S
    tpl = S.build_templates([400, 900, 625], ["sod", "sedov", "sod"], moving=True)
    res, srv = S.run(tpl, rate=3000.0, duration=0.03, steps_per_session=3, keep_final=True)
    assert res["moving"] and res["failed_requests"] == 0
    assert res["requests"] == len(S.I.poisson_arrivals(3000.0, 0.03, 9))
    per_sess = {}
    for r in srv.done:
        per_sess[r.sid] = per_sess.get(r.sid, 0) + 1
    assert srv.used == 0
    moved = 0.0
    for sid, sess in srv.sessions.items():
        ref = _alone_moving(sess.tpl, per_sess[sid])
        assert np.array_equal(sess.final[0], ref[0]) and np.array_equal(sess.final[1], ref[1])
        moved = max(moved, float(np.abs(sess.final[1] - sess.tpl.X0).max()))
    assert moved > 0.0
    assert S.Server.session_bytes(900, True) > S.Server.session_bytes(900)


def _flower_template():
    """A walled box whose central cell has 18 neighbours (a point inside a
    ring of 18), more candidates than a device-rebuilt cell holds (16 slots):
    every device mesh of it is reported, not certified."""
    from paper_1410_3219_amd import inputs as I
    from paper_1410_3219_amd import rich as R
    from paper_1410_3219_amd import serve as S
    from paper_1410_3219_amd import tess as T
    P = I.sod(k=20, seed=4)
    keep = np.hypot(P.px - 0.5, P.py - 0.5) > 0.1
    a = 2 * np.pi * np.arange(18) / 18
    px = np.concatenate([P.px[keep], [0.5], 0.5 + 0.06 * np.cos(a)])
    py = np.concatenate([P.py[keep], [0.5], 0.5 + 0.06 * np.sin(a)])
    m = T.rich_tess_build(px, py, P.box, P.bc)
    deg = np.diff(m.off)
    assert deg.max() >= 18
    n = m.n_cells
    rho = np.where(px < 0.5, 1.0, 0.125)
    pr = np.where(px < 0.5, 1.0, 0.1)
    Q = np.stack([rho * m.area, 0 * m.area, 0 * m.area, pr / (P.gamma - 1) * m.area])
    X = np.stack([m.px, m.py])
    params = R.Params(gamma=P.gamma, motion=1)
    dm = R.DeviceMesh.from_host(m)
    s = R.DeviceState.from_host(Q, X)
    dt = 0.5 * R.rich_cfl_dt(dm, s, params, R.workspace(n))
    return S.Template("flower", n, dm, Q, X, params, dt, s, True), m


def test_served_moving_session_falls_back_to_host_meshes():
    """A session whose device-built meshes are not certified finishes each
    step on host-built meshes, ending in the state the step driver (device
    re-tessellation with the host stage as fallback) reaches."""
    import torch
    from paper_1410_3219_amd import rich as R
    from paper_1410_3219_amd import serve as S
    tpl, m = _flower_template()
    steps = 3
    srv = S.Server([tpl], keep_final=True)
    srv.open_session(0, 0, steps)
    for k in range(steps):
        srv.submit(k, 0, 0.0)
    import time
    t0 = time.perf_counter()
    srv.drain(lambda: time.perf_counter() - t0, timeout_s=120.0)
    assert not srv.failed and srv.fallbacks == steps
    ctx = R.RichCtx(device_tess=True)
    ctx.set_mesh(m)
    st = R.DeviceState.from_host(tpl.Q0, tpl.X0)
    for _ in range(steps):
        ctx.step(st, tpl.dt, tpl.params)
    torch.cuda.synchronize()
    ref = st.numpy()
    assert ctx.tess_counts()[1] == 2 * steps   # every mesh built by the host stage
    ctx.close()
    fin = srv.sessions[0].final
    assert np.array_equal(fin[0], ref[0]) and np.array_equal(fin[1], ref[1])
