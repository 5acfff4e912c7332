"""Cell-rounding parameter sweep (section 6): the Gresho vortex of section
4.3 at 30x30 cells, run for a grid of (chi, eta) values of the rounding
correction, every run advanced together by the batched time-centred step
(rich_step_batch: both stages of all runs as batched launches, the host
tessellations of the runs on parallel host threads).  Reports L of
eq. (Lgresho) for the density of every run.

The end time of the section 6 runs is not stated in the paper; it is a
parameter here.  The analytic density of the vortex is 1 everywhere, so
L = mean_i |rho_i - 1|.

All arithmetic is in the HIP stage kernels and the host tessellation; this
module drives runs and reads results.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs as I
from . import rich as R
from . import tess as T


def chi_eta_grid(n_chi=6, n_eta=6, chi=(0.01, 1.0), eta=(0.001, 0.5)):
    """Log-spaced values over the ranges of section 6, as (chi, eta) pairs."""
    cs = np.exp(np.linspace(math.log(chi[0]), math.log(chi[1]), n_chi))
    es = np.exp(np.linspace(math.log(eta[0]), math.log(eta[1]), n_eta))
    return [(float(c), float(e)) for c in cs for e in es]


class Sweep:
    """device_tess: each run rebuilds its meshes on the device (rich_retess),
    with the host stage only as the fallback for an uncertified mesh."""

    def __init__(self, grid, k=30, seed=4, n_threads=0, device_tess=False):
        P = I.gresho(k=k, seed=seed)
        m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
        self.problem, self.mesh0 = P, m
        self.Q0 = P.state(m.area)
        self.X0 = np.stack([m.px, m.py])
        self.grid = list(grid)
        self.n_threads = n_threads
        self.ctxs, self.states, self.params = [], [], []
        for chi, eta in self.grid:
            c = R.RichCtx(n_threads=1, device_tess=device_tess)
            c.set_mesh(m)
            self.ctxs.append(c)
            self.states.append(R.DeviceState.from_host(self.Q0, self.X0))
            self.params.append(R.Params(gamma=P.gamma, chi=chi, eta=eta, motion=1))
        n = m.n_cells
        self.ws = R.batch_workspace([n] * len(self.grid))
        self.ws_cfl = R.workspace(n)
        self.t = np.zeros(len(self.grid))
        self.steps = np.zeros(len(self.grid), dtype=int)
        self.status = [0] * len(self.grid)

    def live(self):
        return [r for r, s in enumerate(self.status) if s == 0]

    def step(self, dts=None, t_end=None):
        """One time-centred step of every live run (with t_end: of every live
        run not yet at t_end).  dts: per-run time steps (indexed by run),
        else each run's Courant step on the device, clipped so that no run
        passes t_end.  Returns the statuses of the runs stepped."""
        live = self.live()
        if t_end is not None:   # runs already at the end time stay put
            live = [r for r in live if self.t[r] < t_end * (1 - 1e-12)]
        if not live:
            return []
        if dts is None:
            dts = [0.0] * len(self.grid)
            for r in live:
                dts[r] = R.rich_cfl_dt(self.ctxs[r].mesh(), self.states[r], self.params[r],
                                       self.ws_cfl)
        dts = list(dts)
        if t_end is not None:
            for r in live:
                dts[r] = min(dts[r], t_end - self.t[r])
        st = R.rich_step_batch([self.ctxs[r] for r in live], [self.states[r] for r in live],
                               [dts[r] for r in live], [self.params[r] for r in live],
                               self.ws, n_threads=self.n_threads)
        for r, s in zip(live, st):
            if s:
                self.status[r] = s
            else:
                self.t[r] += dts[r]
                self.steps[r] += 1
        return st

    def run(self, t_end, max_steps=100000):
        for _ in range(max_steps):
            if not self.step(t_end=t_end):
                break
        return self

    def density_L(self):
        """eq. (Lgresho) for the density (analytic value 1) of every run;
        the areas come from the host stage on the runs' current points (the
        same tessellation the step driver holds).  NaN for a failed run."""
        P = self.problem
        out = []
        for r in range(len(self.grid)):
            if self.status[r]:
                out.append(float("nan"))
                continue
            Q, X = self.states[r].numpy()
            m = T.rich_tess_build(X[0], X[1], P.box, P.bc)
            rho = Q[0] / m.area
            out.append(float(np.mean(np.abs(rho - 1.0))))
        return out

    def tess_counts(self):
        """(meshes built on the device, meshes the host stage built) over all runs."""
        c = [x.tess_counts() for x in self.ctxs]
        return sum(a for a, _ in c), sum(b for _, b in c)

    def close(self):
        for c in self.ctxs:
            c.close()
        self.ctxs = []
