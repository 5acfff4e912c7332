"""Serving loop (continuous batching of step requests): a session served
among many others ends in exactly the state of the same steps run alone with
single-run stage calls, every request completes, and admission keeps the
device memory of admitted sessions within the budget."""
import numpy as np
import pytest

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
    assert res["mean_batch"] >= 1.0
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
