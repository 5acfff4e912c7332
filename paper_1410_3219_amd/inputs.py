"""Seeded synthetic inputs: mesh-generating points and initial conditions.

This module is the only code shared by the oracle side and the device side.
It holds none of the method's arithmetic: it draws points (splitmix64, so a
C++ port reproduces them bit for bit), samples initial primitive fields at the
points, and converts them to the extensive conserved cell totals that the
method evolves (mass, momentum and total energy integrated over each cell).

Workload recipes (points, box, boundaries, fields) follow the test families
of the paper: the 2D analogue of the shock tube (section 3.3), a point
explosion, the acoustic / advected wave (section 3.2), pure advection
(section 4.1), the Gresho vortex (section 4.3) and the Kelvin-Helmholtz
setup (section 4.4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLD = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start+1 .. start+n of splitmix64 seeded with `seed` (uint64):
    the state advances by the golden-ratio increment and each output is the
    state passed through the two xor-shift-multiply rounds."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLD
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """Doubles in [0, 1): top 53 bits of splitmix64 times 2^-53."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Stream:
    """Sequential uniform draws from one seed (deterministic)."""

    def __init__(self, seed: int):
        self.seed = seed
        self.pos = 0

    def uniform(self, n: int, lo=0.0, hi=1.0) -> np.ndarray:
        z = splitmix64(self.seed, n, self.pos)
        self.pos += n
        u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u


def hilbert_sorted(px, py, box):
    from . import tess
    perm = tess.rich_tess_hilbert_order(px, py, box)
    return px[perm], py[perm]


def jittered_lattice(k: int, seed: int, jitter=0.1, box=(0.0, 0.0, 1.0, 1.0),
                     ky: int | None = None, sort=True):
    """k x ky lattice of cell centres ((i+1/2)h, (j+1/2)h) with per-axis
    uniform jitter in (-jitter*h, +jitter*h)."""
    ky = k if ky is None else ky
    x0, y0, x1, y1 = box
    hx, hy = (x1 - x0) / k, (y1 - y0) / ky
    i, j = np.meshgrid(np.arange(k), np.arange(ky), indexing="ij")
    n = k * ky
    s = Stream(seed)
    jx = s.uniform(n, -jitter, jitter)
    jy = s.uniform(n, -jitter, jitter)
    px = x0 + (i.ravel() + 0.5 + jx) * hx
    py = y0 + (j.ravel() + 0.5 + jy) * hy
    if sort:
        px, py = hilbert_sorted(px, py, box)
    return np.ascontiguousarray(px), np.ascontiguousarray(py)


def uniform_points(n: int, seed: int, box=(0.0, 0.0, 1.0, 1.0), sort=True):
    x0, y0, x1, y1 = box
    s = Stream(seed)
    # keep points strictly inside the box
    px = x0 + (x1 - x0) * (1e-9 + (1 - 2e-9) * s.uniform(n))
    py = y0 + (y1 - y0) * (1e-9 + (1 - 2e-9) * s.uniform(n))
    if sort:
        px, py = hilbert_sorted(px, py, box)
    return np.ascontiguousarray(px), np.ascontiguousarray(py)


def conserved(rho, vx, vy, p, area, gamma):
    """Extensive cell totals (M, Px, Py, E) of uniform primitives on a cell."""
    rho, vx, vy, p, area = (np.broadcast_to(np.asarray(a, dtype=np.float64),
                                            np.shape(area)) for a in (rho, vx, vy, p, area))
    M = rho * area
    E = (p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)) * area
    return np.stack([M, M * vx, M * vy, E]).astype(np.float64)


# --------------------------------------------------------------------------
# Workload recipes.  Each returns (px, py, box, bc, prim(px, py) -> fields).
# --------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    px: np.ndarray
    py: np.ndarray
    box: tuple
    bc: int
    gamma: float
    rho: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    p: np.ndarray
    extra: dict

    @property
    def n(self):
        return int(self.px.shape[0])

    def state(self, area):
        """Q (4, n) on a mesh with cell areas `area`."""
        return conserved(self.rho, self.vx, self.vy, self.p, area, self.gamma)


def sod(k=64, seed=1, gamma=5.0 / 3.0, angle=None, jitter=0.1):
    """2D shock tube: rho=1, p=1 on the left of x=1/2 (or of the line through
    the box centre at `angle`), rho=0.125, p=0.1 on the right; walls."""
    box = (0.0, 0.0, 1.0, 1.0)
    px, py = jittered_lattice(k, seed, jitter, box)
    if angle is None:
        left = px < 0.5
    else:
        left = (px - 0.5) * math.cos(angle) + (py - 0.5) * math.sin(angle) < 0.0
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros_like(px)
    return Problem("sod", px, py, box, 0, gamma, rho, z, z.copy(), p,
                   dict(angle=angle, k=k))


def sedov(k=512, seed=2, gamma=5.0 / 3.0, lloyd_iters=5, e_blast=1.0, n_threads=0):
    """Point explosion: k*k uniform-random points relaxed by Lloyd iterations,
    rho=1, p=1e-6, total energy e_blast added to the cell whose point is
    nearest the box centre (lowest index on a tie); walls."""
    from . import tess
    box = (0.0, 0.0, 1.0, 1.0)
    px, py = uniform_points(k * k, seed, box, sort=True)
    if lloyd_iters:
        px, py = tess.rich_tess_lloyd(px, py, box, 0, lloyd_iters, n_threads)
        px, py = hilbert_sorted(px, py, box)
    d2 = (px - 0.5) ** 2 + (py - 0.5) ** 2
    centre = int(np.argmin(d2))
    n = px.shape[0]
    rho = np.ones(n)
    p = np.full(n, 1e-6)
    z = np.zeros(n)
    return Problem("sedov", px, py, box, 0, gamma, rho, z, z.copy(), p,
                   dict(centre=centre, e_blast=e_blast))


def sedov_state(prob: Problem, area):
    Q = prob.state(area)
    Q[3, prob.extra["centre"]] += prob.extra["e_blast"]
    return Q


def advected_wave(k=2048, seed=3, gamma=5.0 / 3.0, amp=1e-3, v=(1.0, 0.5),
                  p0=0.6, jitter=0.1):
    """rho = 1 + amp sin(2 pi x), uniform p and bulk velocity; periodic."""
    box = (0.0, 0.0, 1.0, 1.0)
    px, py = jittered_lattice(k, seed, jitter, box)
    rho = 1.0 + amp * np.sin(2.0 * np.pi * px)
    n = px.shape[0]
    return Problem("wave", px, py, box, 1, gamma, rho, np.full(n, v[0]),
                   np.full(n, v[1]), np.full(n, p0), dict(amp=amp, v=v))


def acoustic_wave(k=64, seed=3, gamma=5.0 / 3.0, amp=1e-6, v=(0.0, 0.0), jitter=0.1):
    """Linear sound wave: rho = 1 + amp sin(2 pi x), p = 3/5 + amp sin(2 pi x),
    v = bulk (c = 1); periodic."""
    box = (0.0, 0.0, 1.0, 1.0)
    px, py = jittered_lattice(k, seed, jitter, box)
    s = amp * np.sin(2.0 * np.pi * px)
    n = px.shape[0]
    return Problem("acoustic", px, py, box, 1, gamma, 1.0 + s, np.full(n, v[0]) + s,
                   np.full(n, v[1]), 0.6 + s, dict(amp=amp, v=v))


def lattice(k, box=(0.0, 0.0, 1.0, 1.0), ky=None, sort=True):
    """Unjittered lattice of cell centres."""
    return jittered_lattice(k, 0, 0.0, box, ky=ky, sort=sort)


def uniform_flow(k=32, v=(1.0, 0.5), rho=1.0, p=1.0, gamma=5.0 / 3.0, jitter=0.0,
                 seed=5, bc=1):
    box = (0.0, 0.0, 1.0, 1.0)
    px, py = jittered_lattice(k, seed, jitter, box)
    n = px.shape[0]
    return Problem("uniform", px, py, box, bc, gamma, np.full(n, rho),
                   np.full(n, v[0]), np.full(n, v[1]), np.full(n, p), {})


def advection_disc(k=32, gamma=5.0 / 3.0):
    """Pure advection (section 4.1): rho=100 inside r<0.2, 1 outside, p=1,
    v=(1,1), periodic box [-1/2, 1/2]^2, on an unjittered lattice."""
    box = (-0.5, -0.5, 0.5, 0.5)
    px, py = jittered_lattice(k, 0, 0.0, box)
    r = np.hypot(px, py)
    n = px.shape[0]
    return Problem("advection", px, py, box, 1, gamma, np.where(r < 0.2, 100.0, 1.0),
                   np.ones(n), np.ones(n), np.ones(n), {})


def gresho(k=30, seed=4, gamma=5.0 / 3.0, jitter=0.1):
    """Gresho vortex (section 4.3) on [-1/2,1/2]^2, periodic."""
    box = (-0.5, -0.5, 0.5, 0.5)
    px, py = jittered_lattice(k, seed, jitter, box)
    r = np.hypot(px, py)
    p = np.where(r < 0.2, 5 + 12.5 * r * r,
                 np.where(r < 0.4, 9 + 12.5 * r * r - 20 * r + 4 * np.log(np.maximum(5 * r, 1e-300)),
                          3 + 4 * np.log(2.0)))
    vphi = np.where(r < 0.2, 5 * r, np.where(r < 0.4, 2 - 5 * r, 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        cx = np.where(r > 0, -py / r, 0.0)
        cy = np.where(r > 0, px / r, 0.0)
    n = px.shape[0]
    return Problem("gresho", px, py, box, 1, gamma, np.ones(n), vphi * cx, vphi * cy,
                   p, {})


def kelvin_helmholtz(k=50, seed=6, gamma=5.0 / 3.0, jitter=0.1, boost=(0.0, 0.0)):
    """Kelvin-Helmholtz setup (section 4.4), optional constant boost."""
    box = (0.0, 0.0, 1.0, 1.0)
    px, py = jittered_lattice(k, seed, jitter, box)
    inner = np.abs(py - 0.5) < 0.25
    sig = 0.05 / math.sqrt(2.0)
    vy = 0.1 * np.sin(4 * np.pi * px) * (np.exp(-(py - 0.25) ** 2 / (2 * sig * sig)) +
                                        np.exp(-(py - 0.75) ** 2 / (2 * sig * sig)))
    n = px.shape[0]
    return Problem("kh", px, py, box, 1, gamma, np.where(inner, 2.0, 1.0),
                   np.where(inner, 0.5, -0.5) + boost[0], vy + boost[1],
                   np.full(n, 2.5), dict(boost=boost))


def batch_runs(n_runs=256, seed=7, n_min=1024, n_max=65536):
    """Per-run recipes for many independent shock-tube runs of uneven sizes:
    N log-uniform in [n_min, n_max] (lattice side round(sqrt(N))), interface
    angle U[0, pi), gamma U[1.4, 5/3], rounding strength chi U[0, 1]."""
    s = Stream(seed)
    u_n = s.uniform(n_runs)
    u_a = s.uniform(n_runs)
    u_g = s.uniform(n_runs)
    u_c = s.uniform(n_runs)
    runs = []
    for r in range(n_runs):
        N = int(round(math.exp(math.log(n_min) + u_n[r] * (math.log(n_max) - math.log(n_min)))))
        side = max(2, int(round(math.sqrt(N))))
        runs.append(dict(side=side, angle=math.pi * u_a[r],
                         gamma=1.4 + (5.0 / 3.0 - 1.4) * u_g[r], chi=float(u_c[r]),
                         seed=1000 + r))
    return runs


def poisson_arrivals(rate, duration, seed=9):
    """Arrival times of a Poisson process (exponential gaps)."""
    s = Stream(seed)
    t, out = 0.0, []
    while True:
        u = s.uniform(1)[0]
        t += -math.log(1.0 - u) / rate
        if t >= duration:
            return np.array(out)
        out.append(t)
