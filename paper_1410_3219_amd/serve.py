"""Serving loop: continuous batching of time-centred step requests.

Sessions are independent runs whose state lives on the device between
requests.  A request asks for one time-centred step of its session.  The
scheduler:

  * admits a session when the device memory it needs (state buffers, the
    workspace share) fits the HBM budget, otherwise the session waits;
  * on every tick gathers the next stage of every admitted request (stage 1
    of new requests, stage 2 of those whose stage 1 finished) into ONE
    batched launch (rich_stage_batch), so requests that arrive while others
    are on the GPU join the next launch as slots free up;
  * completes a request when its stage 2 finishes and records its latency
    (arrival -> completion event).

Meshes are served from a pool of templates tessellated once by the host
stage and shared read-only by the sessions built on them (static mesh: the
points do not move, so no tessellation happens inside the loop and the
measured latency is the device's).  Every launch is asynchronous; the host
polls completion events.

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


@dataclass
class Request:
    rid: int
    sid: int
    arrival: float
    phase: int = 0          # 0 waiting, 1 stage 1 in flight, 2 stage 2 in flight
    done: float = -1.0


def build_templates(sizes, kinds, seed=11, n_threads=0):
    """One template per (size, kind): host tessellation once, upload once."""
    out = []
    for k, (n, kind) in enumerate(zip(sizes, kinds)):
        side = max(2, int(round(math.sqrt(n))))
        if kind == "sod":
            P = I.sod(k=side, seed=seed + k)
            m = T.rich_tess_build(P.px, P.py, P.box, P.bc, n_threads)
            Q = P.state(m.area)
        else:
            P = I.sedov(k=side, seed=seed + k, lloyd_iters=0)
            m = T.rich_tess_build(P.px, P.py, P.box, P.bc, n_threads)
            Q = I.sedov_state(P, m.area)
        params = R.Params(gamma=P.gamma, motion=0)
        dm = R.DeviceMesh.from_host(m)
        X = np.stack([m.px, m.py])
        s = R.DeviceState.from_host(Q, X)
        ws = R.workspace(m.n_cells)
        dt = R.rich_cfl_dt(dm, s, params, ws)
        out.append(Template(f"{kind}{m.n_cells}", m.n_cells, dm, Q, X, params, 0.5 * dt))
    return out


class Server:
    def __init__(self, templates, hbm_budget_bytes=16 << 30, keep_final=False):
        import torch
        self.torch = torch
        self.templates = templates
        self.budget = hbm_budget_bytes
        self.keep_final = keep_final
        self.used = 0
        self.max_used = 0
        self.sessions = {}
        self.waiting = []          # sessions not yet admitted (FIFO)
        self.queue = []            # requests not yet started
        self.inflight = None       # (event, [(req, stage)], ws)
        self.done = []
        self.launches = 0
        self.batch_sizes = []
        self.cells_done = 0
        self.stream = torch.cuda.current_stream()

    # -- sessions ---------------------------------------------------------
    @staticmethod
    def session_bytes(n):
        # three state buffers (Q: 32 B, X: 16 B per cell) + workspace share
        return 3 * 48 * n + R.rich_workspace_size(n)

    def open_session(self, sid, tpl_index, steps):
        tpl = self.templates[tpl_index]
        s = Session(sid, tpl, steps, bytes=self.session_bytes(tpl.n))
        self.sessions[sid] = s
        self.waiting.append(s)
        return s

    def _admit(self):
        while self.waiting and self.used + self.waiting[0].bytes <= self.budget:
            s = self.waiting.pop(0)
            s.cur = R.DeviceState.from_host(s.tpl.Q0, s.tpl.X0)
            s.half = R.DeviceState.empty_like(s.cur)
            s.nxt = R.DeviceState.empty_like(s.cur)
            s.admitted = True
            self.used += s.bytes
            self.max_used = max(self.max_used, self.used)

    def _close(self, s):
        if self.keep_final:
            s.final = s.cur.numpy()
        s.cur = s.half = s.nxt = None
        s.admitted = False
        self.used -= s.bytes

    # -- requests ---------------------------------------------------------
    def submit(self, rid, sid, arrival):
        self.queue.append(Request(rid, sid, arrival))

    def _launch(self):
        """Gather the ready stages of admitted sessions into one launch."""
        items = []
        busy = set()
        for req in self.queue:
            s = self.sessions[req.sid]
            if not s.admitted or req.sid in busy:
                continue
            busy.add(req.sid)     # one request per session per launch
            items.append(req)
        if not items:
            return False
        meshes, srcs, bases, outs, hs, ps, work = [], [], [], [], [], [], []
        for req in items:
            s = self.sessions[req.sid]
            meshes.append(s.tpl.mesh)
            ps.append(s.tpl.params)
            if req.phase == 0:        # stage 1: (Q^n, Q^n, x^n, dt/2)
                srcs.append(s.cur); bases.append(s.cur); outs.append(s.half)
                hs.append(0.5 * s.tpl.dt)
                work.append((req, 1))
            else:                     # stage 2: (Q^{n+1/2}, Q^n, x^n, dt)
                srcs.append(s.half); bases.append(s.cur); outs.append(s.nxt)
                hs.append(s.tpl.dt)
                work.append((req, 2))
        ws = R.batch_workspace([m.n_cells for m in meshes])
        R.rich_stage_batch(meshes, srcs, bases, outs, hs, ps, ws, self.stream)
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        for req, stage in work:
            req.phase = stage
        self.inflight = (ev, work, ws)
        self.launches += 1
        self.batch_sizes.append(len(work))
        return True

    def _complete(self, now_fn):
        ev, work, ws = self.inflight
        if not ev.query():
            return False
        flags = R.rich_batch_flags(len(work), ws, self.stream)
        t = now_fn()
        for (req, stage), f in zip(work, flags):
            s = self.sessions[req.sid]
            if f:
                raise RuntimeError(f"session {req.sid} stage {stage} flagged {f}")
            if stage == 2:
                s.cur, s.nxt = s.nxt, s.cur
                req.done = t
                self.done.append(req)
                self.queue.remove(req)
                self.cells_done += s.tpl.n
                s.steps_left -= 1
                if s.steps_left == 0:
                    self._close(s)
        self.inflight = None
        return True

    def tick(self, now_fn):
        if self.inflight is not None and not self._complete(now_fn):
            return
        self._admit()
        self._launch()

    def drain(self, now_fn, timeout_s=600.0):
        t0 = time.perf_counter()
        while self.queue or self.inflight is not None:
            self.tick(now_fn)
            if time.perf_counter() - t0 > timeout_s:
                raise RuntimeError("serving loop did not drain")


def run(templates, rate=2000.0, duration=2.0, steps_per_session=8, seed=9,
        hbm_budget_bytes=16 << 30, tpl_choice=None, keep_final=False, log=None):
    """Poisson arrivals of step requests; each session issues its requests in
    order (a session's next request arrives after the previous one).  Returns
    latency percentiles and throughput."""
    import torch
    arrivals = I.poisson_arrivals(rate, duration, seed)
    n_req = len(arrivals)
    n_sess = max(1, n_req // steps_per_session)
    # request k belongs to session k % n_sess, so a session's step count is
    # the number of requests that map to it
    counts = np.bincount(np.arange(n_req) % n_sess, minlength=n_sess)
    s = I.Stream(seed + 1)
    pick = s.uniform(n_sess)
    srv = Server(templates, hbm_budget_bytes, keep_final)
    for sid in range(n_sess):
        ti = tpl_choice[sid] if tpl_choice is not None else int(pick[sid] * len(templates))
        if counts[sid]:
            srv.open_session(sid, ti, int(counts[sid]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0   # noqa: E731
    k = 0
    while k < n_req or srv.queue or srv.inflight is not None:
        t = now()
        while k < n_req and arrivals[k] <= t:
            srv.submit(k, k % n_sess, arrivals[k])
            k += 1
        srv.tick(now)
        if now() > duration * 50 + 120:
            raise RuntimeError("serving run did not finish")
    wall = now()
    lat = np.array([r.done - r.arrival for r in srv.done])
    res = dict(requests=len(srv.done), sessions=n_sess, launches=srv.launches,
               mean_batch=float(np.mean(srv.batch_sizes)) if srv.batch_sizes else 0.0,
               p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
               cell_updates_per_s=srv.cells_done / wall, wall_s=wall, offered_rate=rate,
               hbm_budget_bytes=hbm_budget_bytes, max_admitted_bytes=srv.max_used)
    if log:
        log(f"[serve] {res}")
    return res, srv
