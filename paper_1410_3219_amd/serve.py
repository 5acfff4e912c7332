"""Serving loop: continuous batching of time-centred step requests.

Sessions are independent runs whose state lives on the device between
requests.  A request asks for one time-centred step of its session.  The
scheduler:

  * admits a session when the device memory it needs (state buffers, the
    workspace share) fits the HBM budget, otherwise the session waits;
  * on every tick gathers every ready request (admitted session, none of
    its requests on the device) into one launch pair: stage 1 of all of them
    as one batched launch, then stage 2 as another, back to back on the
    stream; requests that arrive while launches are on the device join the
    next pair, and up to two pairs are in flight at once;
  * completes the requests of a pair when its event has passed, checks the
    per-run flags and records each latency (arrival -> completion);
  * evicts a session whose step is flagged (negative density or pressure,
    a point outside the domain): the failed step is not committed, the
    session's device memory is released, its request and every later one
    of that session complete as failed, and the other sessions of the same
    launch, which the batched stage keeps independent, go on unaffected.

Meshes are served from a pool of templates tessellated once by the host
stage and shared read-only by the sessions built on them.  With static
templates the points do not move, so no tessellation happens inside the
loop and the measured latency is the device's.  With moving templates
(Lagrangian motion) each session's mesh is rebuilt on the device twice per
step, batched over the launch's sessions: stage 1, re-tessellation of the
half-step points, stage 2 on that mesh, re-tessellation of the new points;
each session keeps three mesh buffers in rotation and a re-tessellation
workspace.  A step whose device-built mesh is not certified is redone for
that session with the host stage (as the step driver does), at host speed;
the loop counts such steps.  Launches are asynchronous, the batched
re-tessellation's included (its descriptors go through the library's pinned
staging ring, and its flags come back with the launch's flag words); the
host polls completion events.

All arithmetic is in the batched HIP stage; this module only schedules.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I
from . import rich as R
from . import tess as T


@dataclass
class Template:
    name: str
    n: int
    mesh: "R.DeviceMesh"
    Q0: np.ndarray
    X0: np.ndarray
    params: "R.Params"
    dt: float
    state0: "R.DeviceState" = None   # initial state on the device (copied per session)
    moving: bool = False             # Lagrangian motion: meshes rebuilt on the device


@dataclass
class Session:
    sid: int
    tpl: Template
    steps_left: int
    cur: "R.DeviceState" = None
    half: "R.DeviceState" = None
    nxt: "R.DeviceState" = None
    admitted: bool = False
    bytes: int = 0
    final: tuple = None     # (Q, X) on the host at close, when kept
    error: int = 0          # stage flags (stage 1 | stage 2 << 8; 1 << 16: a mesh
                            # not certified) of an evicted session
    mesh: "R.DeviceMesh" = None     # moving: the current mesh
    mbufs: list = None              # moving: three mesh buffers in rotation
    rws: object = None              # moving: re-tessellation workspace
    b: int = 0                      # moving: rotation index


@dataclass
class Request:
    rid: int
    sid: int
    arrival: float
    phase: int = 0          # 0 waiting, 1 on the device
    done: float = -1.0
    failed: bool = False


def build_templates(sizes, kinds, seed=11, n_threads=0, moving=False):
    """One template per (size, kind): host tessellation once, upload once;
    moving: Lagrangian motion with cell rounding (the paper's defaults),
    else a static mesh."""
    out = []
    for k, (n, kind) in enumerate(zip(sizes, kinds)):
        side = max(2, int(round(math.sqrt(n))))
        if kind == "sod":
            P = I.sod(k=side, seed=seed + k)
            m = T.rich_tess_build(P.px, P.py, P.box, P.bc, n_threads)
            Q = P.state(m.area)
        else:
            # moving meshes start from Lloyd-relaxed points (regular cells)
            P = I.sedov(k=side, seed=seed + k, lloyd_iters=5 if moving else 0)
            m = T.rich_tess_build(P.px, P.py, P.box, P.bc, n_threads)
            Q = I.sedov_state(P, m.area)
        params = R.Params(gamma=P.gamma, motion=1 if moving else 0)
        dm = R.DeviceMesh.from_host(m)
        X = np.stack([m.px, m.py])
        s = R.DeviceState.from_host(Q, X)
        ws = R.workspace(m.n_cells)
        dt = R.rich_cfl_dt(dm, s, params, ws)
        out.append(Template(f"{kind}{m.n_cells}", m.n_cells, dm, Q, X, params, 0.5 * dt, s,
                            moving))
    return out


class Server:
    """Continuous batching of step requests over device-resident sessions.

    A launch takes every request that is ready (session admitted, no other
    request of the same session on the device) and issues both stages of its
    step back to back as two batched launches on one stream, so stage 2 needs
    no host round trip; up to `max_inflight` such launch pairs are on the
    device at once, each with its own workspaces, while the host gathers the
    next.  With moving templates each stage is followed by a batched
    re-tessellation, enqueued the same way.  Sessions are admitted in arrival order while
    their device memory fits the budget and released when their last request
    completes."""

    def __init__(self, templates, hbm_budget_bytes=16 << 30, keep_final=False,
                 max_inflight=2):
        import torch
        self.torch = torch
        self.templates = templates
        self.moving = any(t.moving for t in templates)
        if self.moving and not all(t.moving for t in templates):
            raise ValueError("templates are either all moving or all static")
        self.budget = hbm_budget_bytes
        self.keep_final = keep_final
        # the batched re-tessellation waits on the stream: one pair in flight
        self.max_inflight = max_inflight
        self.used = 0
        self.max_used = 0
        self.sessions = {}
        self.waiting = []          # sessions not yet admitted (FIFO)
        self.queue = []            # requests not yet completed, in arrival order
        self.inflight = []         # [(event, [req], ws1, ws2, host flags, retess workspaces)]
        self.ws_pool = []          # idle batch workspaces
        self.busy = set()          # sessions with a request on the device
        self.done = []
        self.failed = []           # requests of evicted sessions
        self.fallbacks = 0         # moving: steps redone with host-built meshes
        self.launches = 0
        self.batch_sizes = []
        self.launch_templates = []   # per launch: the sorted template indices it carried
        self._tpl_index = {id(t): k for k, t in enumerate(templates)}
        self.cells_done = 0
        self.stream = torch.cuda.current_stream()

    # -- sessions ---------------------------------------------------------
    @staticmethod
    def session_bytes(n, moving=False):
        # three state buffers (Q: 32 B, X: 16 B per cell) and the session's
        # share of the two workspaces of its launch pair; moving: three mesh
        # buffers at capacity and a re-tessellation workspace
        b = 3 * 48 * n + 2 * R.rich_workspace_size(n)
        if moving:
            ce, cc = R.rich_retess_capacity(n)
            mesh = R.CELL_BYTES * n + R.EDGE_BYTES * ce + 8 * (n + 1) + 4 * cc
            b += 3 * mesh + R.rich_retess_workspace_size(n)
        return b

    def _ws(self, n_cells):
        """A batch workspace for these runs from the pool of idle ones (the
        smallest that fits), else a new one with 25 % headroom."""
        need = R.rich_batch_workspace_size(n_cells)
        fit = [k for k, w in enumerate(self.ws_pool) if w.numel() >= need]
        if fit:
            k = min(fit, key=lambda j: self.ws_pool[j].numel())
            return self.ws_pool.pop(k)
        import torch
        return torch.empty(need + need // 4, dtype=torch.uint8, device="cuda")

    def open_session(self, sid, tpl_index, steps):
        tpl = self.templates[tpl_index]
        s = Session(sid, tpl, steps, bytes=self.session_bytes(tpl.n, tpl.moving))
        self.sessions[sid] = s
        self.waiting.append(s)
        return s

    def _admit(self):
        while self.waiting and self.used + self.waiting[0].bytes <= self.budget:
            s = self.waiting.pop(0)
            t0 = s.tpl.state0
            if t0 is not None:   # device-to-device copy of the template's state
                s.cur = R.DeviceState(t0.Q.clone(), t0.X.clone())
            else:
                s.cur = R.DeviceState.from_host(s.tpl.Q0, s.tpl.X0)
            s.half = R.DeviceState.empty_like(s.cur)
            s.nxt = R.DeviceState.empty_like(s.cur)
            if s.tpl.moving:
                m = s.tpl.mesh
                s.mesh = m
                s.mbufs = [R.DeviceMeshBufs(m.n_cells, m.box, m.bc) for _ in range(3)]
                s.rws = R.retess_workspace(m.n_cells)
                s.b = 0
            s.admitted = True
            self.used += s.bytes
            self.max_used = max(self.max_used, self.used)

    def _close(self, s):
        if self.keep_final:
            s.final = s.cur.numpy()
        s.cur = s.half = s.nxt = None
        s.mesh = s.mbufs = s.rws = None
        s.admitted = False
        self.used -= s.bytes

    def _evict(self, s, flags, t):
        """Close a session whose step was flagged; its committed state (the
        one before the failed step) is what keep_final records."""
        s.error = flags
        self.busy.discard(s.sid)
        self._close(s)
        for req in self.queue:
            if req.sid == s.sid and req.done < 0:
                req.done, req.failed = t, True
                self.failed.append(req)

    # -- requests ---------------------------------------------------------
    def submit(self, rid, sid, arrival):
        req = Request(rid, sid, arrival)
        if self.sessions[sid].error:   # evicted: fails at once
            req.done, req.failed = arrival, True
            self.failed.append(req)
            return
        self.queue.append(req)

    def _launch(self):
        items = []
        seen = set()
        for req in self.queue:
            s = self.sessions[req.sid]
            if req.phase or not s.admitted or req.sid in self.busy or req.sid in seen:
                continue
            seen.add(req.sid)     # a session's requests run in order
            items.append(req)
        if not items:
            return False
        ss = [self.sessions[r.sid] for r in items]
        meshes = [s.tpl.mesh for s in ss]
        ps = [s.tpl.params for s in ss]
        ns = [m.n_cells for m in meshes]
        ws1, ws2 = self._ws(ns), self._ws(ns)
        rt = None
        if self.moving:
            meshes = [s.mesh for s in ss]
            hb = [s.mbufs[s.b % 3] for s in ss]
            nb = [s.mbufs[(s.b + 1) % 3] for s in ss]
            hmeshes = [b.mesh() for b in hb]
        else:
            hmeshes = meshes
        # stage 1: (Q^n, Q^n, x^n, dt/2) -> half; stage 2: (half, Q^n, x^n, dt) -> nxt,
        # on the mesh of the half-step points when the points move
        R.rich_stage_batch(meshes, [s.cur for s in ss], [s.cur for s in ss],
                           [s.half for s in ss], [0.5 * s.tpl.dt for s in ss], ps, ws1,
                           self.stream)
        if self.moving:
            bws1 = R.rich_retess_batch(meshes, [s.half.X for s in ss], hb,
                                       [s.rws for s in ss], stream=self.stream)
        R.rich_stage_batch(hmeshes, [s.half for s in ss], [s.cur for s in ss],
                           [s.nxt for s in ss], [s.tpl.dt for s in ss], ps, ws2, self.stream)
        if self.moving:
            bws2 = R.rich_retess_batch(hmeshes, [s.nxt.X for s in ss], nb,
                                       [s.rws for s in ss], stream=self.stream)
            # both meshes' flags come back with the launch as well
            mflags = self.torch.empty((2, len(items)), dtype=self.torch.int32, pin_memory=True)
            R.rich_retess_batch_flags_async(len(items), bws1, mflags[0], self.stream)
            R.rich_retess_batch_flags_async(len(items), bws2, mflags[1], self.stream)
            rt = (bws1, bws2, mflags)
        # both stages' flag words come back with the launch (no stream sync)
        flags = self.torch.empty((2, len(items)), dtype=self.torch.int32, pin_memory=True)
        R.rich_batch_flags_async(len(items), ws1, flags[0], self.stream)
        R.rich_batch_flags_async(len(items), ws2, flags[1], self.stream)
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        for r in items:
            r.phase = 1
            self.busy.add(r.sid)
        self.inflight.append((ev, items, ws1, ws2, flags, rt))
        self.launches += 1
        self.batch_sizes.append(len(items))
        self.launch_templates.append(tuple(sorted({self._tpl_index[id(s.tpl)] for s in ss})))
        return True

    def _complete(self, now_fn):
        progressed = False
        while self.inflight and self.inflight[0][0].query():
            ev, items, ws1, ws2, flags, rt = self.inflight.pop(0)
            f1, f2 = flags[0].tolist(), flags[1].tolist()
            half_ok = [True] * len(items)
            new_ok = [True] * len(items)
            if rt is not None:   # both meshes of each session's step (their flags)
                half_ok = [f == 0 for f in rt[2][0].tolist()]
                new_ok = [f == 0 for f in rt[2][1].tolist()]
            self.ws_pool += [ws1, ws2]
            if len(self.ws_pool) > 4 * self.max_inflight:   # keep the largest idle ones
                self.ws_pool.sort(key=lambda t: t.numel())
                del self.ws_pool[:len(self.ws_pool) - 4 * self.max_inflight]
            t = now_fn()
            for req, a, b, h_ok, n_ok in zip(items, f1, f2, half_ok, new_ok):
                s = self.sessions[req.sid]
                # stage 2 counts only on a certified half-step mesh
                if a or (h_ok and b):
                    self._evict(s, (a & 0xff) | ((b & 0xff) << 8), t)
                    continue
                if self.moving:
                    if h_ok and n_ok:
                        s.mesh = s.mbufs[(s.b + 1) % 3].mesh()
                    else:
                        f = self._host_step(s, h_ok)
                        if f:
                            self._evict(s, (f & 0xff) << 8, t)
                            continue
                        self.fallbacks += 1
                    s.b += 2
                s.cur, s.nxt = s.nxt, s.cur
                req.done = t
                self.done.append(req)
                self.busy.discard(req.sid)
                self.cells_done += s.tpl.n
                s.steps_left -= 1
                if s.steps_left == 0:
                    self._close(s)
            progressed = True
        if progressed:   # one pass over the queue per completion, not per request
            self.queue = [r for r in self.queue if r.done < 0]
        return progressed

    def _host_step(self, s, half_ok):
        """Finish session s's step with host-built meshes: stage 1 ran on its
        certified current mesh; if the half-step mesh was not certified,
        stage 2 is redone on the host stage's mesh of the half-step points;
        the new mesh is the host stage's.  Returns stage 2's flags."""
        from . import tess as T
        m = s.mesh
        flags = 0
        if not half_ok:
            xh = s.half.X.cpu().numpy()
            hm = R.DeviceMesh.from_host(T.rich_tess_build(xh[0], xh[1], m.box, m.bc))
            ws = R.workspace(s.tpl.n)
            R.rich_stage(hm, s.half, s.cur, s.nxt, s.tpl.dt, s.tpl.params, ws, self.stream)
            flags = R.rich_stage_flags(ws, self.stream)
            if flags:
                return flags
        xn = s.nxt.X.cpu().numpy()
        s.mesh = R.DeviceMesh.from_host(T.rich_tess_build(xn[0], xn[1], m.box, m.bc))
        return flags

    def tick(self, now_fn):
        self._complete(now_fn)
        self._admit()
        if len(self.inflight) < self.max_inflight:
            self._launch()

    def drain(self, now_fn, timeout_s=600.0):
        t0 = time.perf_counter()
        while self.queue or self.inflight:
            self.tick(now_fn)
            if time.perf_counter() - t0 > timeout_s:
                raise RuntimeError("serving loop did not drain")


def run(templates, rate=2000.0, duration=2.0, steps_per_session=8, seed=9,
        hbm_budget_bytes=16 << 30, tpl_choice=None, keep_final=False, max_inflight=2,
        log=None):
    """Poisson arrivals of step requests; requests k*S .. k*S+S-1 (S =
    steps_per_session) are the steps of session k, which opens when its
    first request arrives.  Returns latency percentiles (arrival ->
    completion seen by the host) and throughput."""
    import torch
    arrivals = I.poisson_arrivals(rate, duration, seed)
    n_req = len(arrivals)
    n_sess = max(1, (n_req + steps_per_session - 1) // steps_per_session)
    s = I.Stream(seed + 1)
    pick = s.uniform(n_sess)
    srv = Server(templates, hbm_budget_bytes, keep_final, max_inflight)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0   # noqa: E731
    k = 0
    while k < n_req or srv.queue or srv.inflight:
        t = now()
        while k < n_req and arrivals[k] <= t:
            sid = k // steps_per_session
            if k % steps_per_session == 0:
                ti = (tpl_choice[sid] if tpl_choice is not None
                      else int(pick[sid] * len(templates)))
                srv.open_session(sid, ti, min(steps_per_session, n_req - k))
            srv.submit(k, sid, arrivals[k])
            k += 1
        srv.tick(now)
        if now() > duration * 50 + 120:
            raise RuntimeError("serving run did not finish")
    wall = now()
    lat = np.array([r.done - r.arrival for r in srv.done]) if srv.done else np.zeros(1)
    res = dict(moving=srv.moving, host_fallback_steps=srv.fallbacks,
               requests=len(srv.done), failed_requests=len(srv.failed),
               evicted_sessions=sum(1 for x in srv.sessions.values() if x.error),
               sessions=n_sess, launches=srv.launches,
               mean_batch=float(np.mean(srv.batch_sizes)) if srv.batch_sizes else 0.0,
               max_batch=int(max(srv.batch_sizes)) if srv.batch_sizes else 0,
               mixed_launches=sum(1 for t in srv.launch_templates if len(t) > 1),
               p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
               cell_updates_per_s=srv.cells_done / wall, wall_s=wall, offered_rate=rate,
               offered_cell_updates_per_s=rate * float(np.mean([t.n for t in templates])),
               hbm_budget_bytes=hbm_budget_bytes, max_admitted_bytes=srv.max_used)
    if log:
        log(f"[serve] {res}")
    return res, srv
