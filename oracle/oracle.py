"""ctypes wrapper of the plain serial FP64 oracle (liboracle.so, oracle.h).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use this module; the product path never does.  It imports
nothing from the device-side package: meshes are any objects carrying the
host-stage arrays (px, py, sx, sy, area, e_i, e_j, e_len, e_fx, e_fy, off,
idx, box, bc), and the time-centred step takes the tessellation as a callable.

or_step composes two stages the way section 2.3 of the paper describes the
"time centred fluxes" scheme: advance half a step, rebuild the mesh from the
half-step points, compute the primitives there, apply the resulting fluxes
to the start-of-step state with the full step, and move the points from their
start-of-step positions with the half-step point velocities.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


OMP_LIB_PATH = os.path.join(_HERE, "liboracle_omp.so")
FMA_LIB_PATH = os.path.join(_HERE, "liboracle_fma.so")


def build(force=False):
    """Compile liboracle.so with gcc (plain C99, -O2, no FMA contraction),
    the reference build; liboracle_omp.so, the same source with its per-cell
    and per-edge loops spread over OpenMP threads (only for timing the
    oracle on all host cores); and liboracle_fma.so, the same source with
    fused multiply-adds, which rounds differently (only for measuring how
    much a long chain amplifies rounding differences)."""
    fp_off = ["-ffp-contract=off"]
    for path, extra in ((LIB_PATH, fp_off), (OMP_LIB_PATH, fp_off + ["-fopenmp"]),
                        (FMA_LIB_PATH, ["-mfma", "-ffp-contract=fast"])):
        if force or not os.path.exists(path) or \
                os.path.getmtime(path) < os.path.getmtime(SRC_PATH):
            cmd = ["gcc", "-O2", "-std=c99", *extra, "-fPIC", "-shared",
                   SRC_PATH, "-o", path + ".tmp", "-lm"]
            subprocess.check_call(cmd)
            os.replace(path + ".tmp", path)
    return LIB_PATH


def threads():
    """Threads the loaded build runs its loops on (1 for the reference)."""
    return int(lib().or_threads())


class OrMesh(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int64), ("n_edges", C.c_int64),
        ("px", _dp), ("py", _dp), ("sx", _dp), ("sy", _dp), ("area", _dp),
        ("e_i", _ip), ("e_j", _ip), ("e_len", _dp), ("e_fx", _dp), ("e_fy", _dp),
        ("off", _ip), ("idx", _ip), ("box", C.c_double * 4), ("bc", C.c_uint32),
    ]


class OrParams(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("cfl", C.c_double), ("theta", C.c_double),
        ("delta_v", C.c_double), ("delta_p", C.c_double), ("chi", C.c_double),
        ("eta", C.c_double), ("riemann", C.c_int32), ("motion", C.c_int32),
        ("limiter", C.c_int32), ("gx", C.c_double), ("gy", C.c_double),
        ("integrator", C.c_int32),
    ]


@dataclass
class Params:
    """Scheme parameters; defaults are the paper's (sections 2.2, 2.3, 6)."""
    gamma: float = 5.0 / 3.0
    cfl: float = 0.3
    theta: float = 0.5
    delta_v: float = 0.2
    delta_p: float = 0.7
    chi: float = 0.15
    eta: float = 0.02
    riemann: int = 0   # 0 HLLC, 1 exact
    motion: int = 1    # 0 static, 1 Lagrangian + cell rounding
    limiter: int = 0   # 0 switching, 1 global, 2 local, 3 unlimited, 4 first order
    gx: float = 0.0    # uniform external acceleration
    gy: float = 0.0
    integrator: int = 0   # 0 time-centred fluxes, 1 extrapolated fluxes

    def c(self):
        return OrParams(self.gamma, self.cfl, self.theta, self.delta_v, self.delta_p,
                        self.chi, self.eta, self.riemann, self.motion, self.limiter,
                        self.gx, self.gy, self.integrator)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        mp, pp = C.POINTER(OrMesh), C.POINTER(OrParams)
        L.or_primitives.argtypes = [mp, _dp, pp, _dp]
        L.or_point_velocity.argtypes = [mp, _dp, pp, _dp]
        L.or_gradients.argtypes = [mp, _dp, _dp]
        L.or_limiter.argtypes = [mp, _dp, _dp, pp, _dp, _ip]
        L.or_edge_fluxes.argtypes = [mp, _dp, _dp, _dp, pp, _dp]
        L.or_edge_waves.argtypes = [mp, _dp, _dp, _dp, pp, _dp]
        L.or_area_rate.argtypes = [mp, _dp, _dp]
        L.or_stage.argtypes = [mp, _dp, _dp, _dp, C.c_double, pp, _dp, _dp, _dp, _dp,
                               _dp, _ip, _dp]
        L.or_cfl_dt.argtypes = [mp, _dp, pp, _dp]
        L.or_stage_accel.argtypes = [mp, _dp, _dp, _dp, C.c_double, pp, _dp, _dp, _dp, _dp]
        L.or_voronoi.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_uint32, C.c_int32, _dp, _dp,
                                 _dp, _ip, _ip, _dp, _dp, _dp]
        L.or_hllc.argtypes = [C.c_double, _dp, _dp, _dp]
        L.or_hllc.restype = None
        L.or_exact.argtypes = [C.c_double, _dp, _dp, _dp, _dp]
        L.or_exact_sample.argtypes = [C.c_double, _dp, _dp, C.c_double, _dp]
        for f in ("or_primitives", "or_point_velocity", "or_gradients", "or_limiter",
                  "or_edge_fluxes", "or_edge_waves", "or_area_rate", "or_stage", "or_stage_accel",
                  "or_cfl_dt", "or_exact",
                  "or_exact_sample", "or_voronoi"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class _MeshRef:
    """Keeps the contiguous arrays alive while the C struct points at them."""

    def __init__(self, mesh):
        self.a = {}
        for k in ("px", "py", "sx", "sy", "area", "e_len", "e_fx", "e_fy"):
            self.a[k] = np.ascontiguousarray(getattr(mesh, k), dtype=np.float64)
        for k in ("e_i", "e_j", "off", "idx"):
            self.a[k] = np.ascontiguousarray(getattr(mesh, k), dtype=np.int32)
        self.n = self.a["px"].shape[0]
        self.ne = self.a["e_i"].shape[0]
        self.s = OrMesh(self.n, self.ne,
                        *[_d(self.a[k]) for k in ("px", "py", "sx", "sy", "area")],
                        _i(self.a["e_i"]), _i(self.a["e_j"]),
                        *[_d(self.a[k]) for k in ("e_len", "e_fx", "e_fy")],
                        _i(self.a["off"]), _i(self.a["idx"]),
                        (C.c_double * 4)(*mesh.box), int(mesh.bc))


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == shape, (a.shape, shape)
    return a


def primitives(mesh, Q, p: Params):
    m = _MeshRef(mesh)
    Q = _f64(Q, (4, m.n))
    out = np.empty((5, m.n))
    lib().or_primitives(C.byref(m.s), _d(Q), C.byref(p.c()), _d(out))
    return out


def point_velocity(mesh, prim, p: Params):
    m = _MeshRef(mesh)
    prim = _f64(prim, (5, m.n))
    w = np.empty((2, m.n))
    lib().or_point_velocity(C.byref(m.s), _d(prim), C.byref(p.c()), _d(w))
    return w


def gradients(mesh, prim):
    """Unlimited gradients (8, n): d/dx, d/dy of rho, vx, vy, p."""
    m = _MeshRef(mesh)
    prim = _f64(prim, (5, m.n))
    g = np.empty((8, m.n))
    lib().or_gradients(C.byref(m.s), _d(prim), _d(g))
    return g


def limiter(mesh, prim, grad, p: Params):
    m = _MeshRef(mesh)
    prim = _f64(prim, (5, m.n))
    grad = _f64(grad, (8, m.n))
    alpha = np.empty((4, m.n))
    flag = np.empty(m.n, dtype=np.int32)
    lib().or_limiter(C.byref(m.s), _d(prim), _d(grad), C.byref(p.c()), _d(alpha),
                     _i(flag))
    return alpha, flag


def edge_fluxes(mesh, prim, lgrad, w, p: Params):
    m = _MeshRef(mesh)
    prim, lgrad, w = _f64(prim, (5, m.n)), _f64(lgrad, (8, m.n)), _f64(w, (2, m.n))
    F = np.empty((4, m.ne))
    st = lib().or_edge_fluxes(C.byref(m.s), _d(prim), _d(lgrad), _d(w), C.byref(p.c()),
                              _d(F))
    return F, st


def edge_waves(mesh, prim, lgrad, w, p: Params):
    """(4, E): the quantities whose signs pick the Riemann solver's branch
    on each edge (HLLC: S_L, S*, S_R; exact: NaN, u*, NaN) and a velocity
    scale of the edge's two states."""
    m = _MeshRef(mesh)
    prim, lgrad, w = _f64(prim, (5, m.n)), _f64(lgrad, (8, m.n)), _f64(w, (2, m.n))
    out = np.empty((4, m.ne))
    st = lib().or_edge_waves(C.byref(m.s), _d(prim), _d(lgrad), _d(w), C.byref(p.c()),
                             _d(out))
    return out, st


def area_rate(mesh, w):
    m = _MeshRef(mesh)
    w = _f64(w, (2, m.n))
    out = np.empty(m.n)
    lib().or_area_rate(C.byref(m.s), _d(w), _d(out))
    return out


@dataclass
class StageResult:
    Q: np.ndarray
    X: np.ndarray
    status: int
    prim: np.ndarray = None
    w: np.ndarray = None
    alpha: np.ndarray = None
    flag: np.ndarray = None
    flux: np.ndarray = None


def stage(mesh, Qsrc, Qbase, Xbase, h, p: Params, diag=False) -> StageResult:
    """One stage (mesh, Q_src, Q_base, X_base, h) -> (Q_out, X_out)."""
    m = _MeshRef(mesh)
    Qsrc, Qbase = _f64(Qsrc, (4, m.n)), _f64(Qbase, (4, m.n))
    Xbase = _f64(Xbase, (2, m.n))
    Qout = np.empty((4, m.n))
    Xout = np.empty((2, m.n))
    if diag:
        prim, w = np.empty((5, m.n)), np.empty((2, m.n))
        alpha, flag = np.empty((4, m.n)), np.empty(m.n, dtype=np.int32)
        flux = np.empty((4, max(m.ne, 1)))
        ptrs = (_d(prim), _d(w), _d(alpha), _i(flag), _d(flux))
    else:
        prim = w = alpha = flag = flux = None
        ptrs = (None, None, None, None, None)
    st = lib().or_stage(C.byref(m.s), _d(Qsrc), _d(Qbase), _d(Xbase), float(h),
                        C.byref(p.c()), _d(Qout), _d(Xout), *ptrs)
    if diag:
        flux = flux[:, :m.ne]
    return StageResult(Qout, Xout, st, prim, w, alpha, flag, flux)


def stage_accel(mesh, Qsrc, Qbase, Xbase, h, p: Params, accel) -> StageResult:
    """One stage with a per-cell external acceleration accel (2, n) added to
    the uniform one of p."""
    m = _MeshRef(mesh)
    Qsrc, Qbase = _f64(Qsrc, (4, m.n)), _f64(Qbase, (4, m.n))
    Xbase = _f64(Xbase, (2, m.n))
    a = _f64(accel, (2, m.n))
    Qout = np.empty((4, m.n))
    Xout = np.empty((2, m.n))
    ax, ay = np.ascontiguousarray(a[0]), np.ascontiguousarray(a[1])
    st = lib().or_stage_accel(C.byref(m.s), _d(Qsrc), _d(Qbase), _d(Xbase), float(h),
                              C.byref(p.c()), _d(ax), _d(ay), _d(Qout), _d(Xout))
    return StageResult(Qout, Xout, st, None, None, None, None, None)


def cfl_dt(mesh, Q, p: Params):
    m = _MeshRef(mesh)
    Q = _f64(Q, (4, m.n))
    dt = C.c_double(0.0)
    st = lib().or_cfl_dt(C.byref(m.s), _d(Q), C.byref(p.c()), C.byref(dt))
    return dt.value, st


def hllc(gamma, WL, WR):
    WL, WR = (np.ascontiguousarray(v, dtype=np.float64) for v in (WL, WR))
    F = np.empty(4)
    lib().or_hllc(float(gamma), _d(WL), _d(WR), _d(F))
    return F


def exact(gamma, WL, WR):
    """(flux at x/t=0, p*, u*, iterations)."""
    WL, WR = (np.ascontiguousarray(v, dtype=np.float64) for v in (WL, WR))
    F, star = np.empty(4), np.empty(2)
    it = lib().or_exact(float(gamma), _d(WL), _d(WR), _d(F), _d(star))
    return F, star[0], star[1], it


def exact_sample(gamma, WL, WR, xi):
    WL, WR = (np.ascontiguousarray(v, dtype=np.float64) for v in (WL, WR))
    W = np.empty(4)
    it = lib().or_exact_sample(float(gamma), _d(WL), _d(WR), float(xi), _d(W))
    return W, it


def step(mesh, Q, X, dt, p: Params, tess, diag=False, accel=None):
    """One step (section 2.3).  `tess(px, py, box, bc)` returns the mesh of
    the given points.  Returns (Q_new, X_new, mesh_new, mesh_half, status).
    accel (2, n): a per-cell acceleration added to p's uniform one in every
    stage (cells keep their index through the step).

    Time-centred fluxes (integrator 0): a half stage, the mesh rebuilt, then
    the full stage from the start-of-step state with the half-step fluxes.
    Extrapolated fluxes (integrator 1): one full stage on the start-of-step
    mesh with half-step face states, the points moved by dt w^n."""
    def st(m, Qs, Qb, Xb, h):
        return stage(m, Qs, Qb, Xb, h, p) if accel is None else \
            stage_accel(m, Qs, Qb, Xb, h, p, accel)

    if p.integrator == 1:
        s = st(mesh, Q, Q, X, dt)
        if s.status != 0:
            return None, None, None, None, s.status
        mesh_n = tess(s.X[0], s.X[1], mesh.box, mesh.bc) if p.motion else mesh
        return s.Q, s.X, mesh_n, None, 0
    s1 = st(mesh, Q, Q, X, 0.5 * dt)
    if s1.status != 0:
        return None, None, None, None, s1.status
    mesh_h = tess(s1.X[0], s1.X[1], mesh.box, mesh.bc) if p.motion else mesh
    s2 = st(mesh_h, s1.Q, Q, X, dt)
    if s2.status != 0:
        return None, None, None, mesh_h, s2.status
    mesh_n = tess(s2.X[0], s2.X[1], mesh.box, mesh.bc) if p.motion else mesh
    return s2.Q, s2.X, mesh_n, mesh_h, 0


class use_library:
    """Context manager: route this module's calls to another build of the
    oracle (used by the test that plants mistakes in a copy of oracle.c)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = None
        saved_path = LIB_PATH
        globals()["LIB_PATH"] = self.path
        try:
            lib()
        finally:
            globals()["LIB_PATH"] = saved_path
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def build_variant(src_text, out_path, fp_flags=("-ffp-contract=off",)):
    """Compile oracle source text (a modified copy) to out_path.  fp_flags
    replaces the default floating-point flags (the tests of the parity
    metric build the unmodified source with fused multiply-adds)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", *fp_flags, "-fPIC",
                           "-shared", "-I", _HERE, src, "-o", out_path, "-lm"])
    return out_path


# ---------------------------------------------------------------------------
# Voronoi mesh by definition (input stage, section 2.1)
# ---------------------------------------------------------------------------
CELL_MASK = 0x0FFFFFFF
CODE_SHIFT = 28


class Voronoi:
    """Cells of or_voronoi: area, centroid (sx, sy) and, per cell, the
    counter-clockwise list of (neighbour cell, code, length, midpoint)."""


def voronoi(px, py, box, bc, max_fan=32):
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    n = px.shape[0]
    bx = np.ascontiguousarray(box, dtype=np.float64)
    V = Voronoi()
    V.px, V.py, V.box, V.bc, V.max_fan = px, py, tuple(box), int(bc), max_fan
    V.area, V.sx, V.sy = np.empty(n), np.empty(n), np.empty(n)
    V.deg = np.zeros(n, dtype=np.int32)
    V.nb = np.zeros(n * max_fan, dtype=np.int32)
    V.len, V.fx, V.fy = (np.zeros(n * max_fan) for _ in range(3))
    st = lib().or_voronoi(n, _d(px), _d(py), _d(bx), int(bc), max_fan, _d(V.area), _d(V.sx),
                          _d(V.sy), _i(V.deg), _i(V.nb), _d(V.len), _d(V.fx), _d(V.fy))
    if st != 0:
        raise ValueError(f"or_voronoi failed ({st})")
    return V


def fan(V, i):
    """[(cell, code, length, fx, fy)] of cell i, counter-clockwise."""
    out = []
    for q in range(V.deg[i]):
        s = i * V.max_fan + q
        u = int(V.nb[s]) & 0xFFFFFFFF
        out.append((u & CELL_MASK, u >> CODE_SHIFT, V.len[s], V.fx[s], V.fy[s]))
    return out


def voronoi_mesh(V):
    """The mesh arrays of the input stage (px, py, sx, sy, area, e_i, e_j,
    e_len, e_fx, e_fy, off, idx, box, bc) assembled from the cells: an edge
    belongs to the lower-numbered cell (a wall edge to its cell, an edge
    between a cell and its own periodic image to the side with code >= 5);
    each cell's CSR lists its edges counter-clockwise as 2 * edge + side."""
    n = V.px.shape[0]

    def owns(i, cell, code):
        if code >= 9:
            return True
        if cell != i:
            return i < cell
        return code >= 5

    e_i, e_j, e_len, e_fx, e_fy, where = [], [], [], [], [], {}
    for i in range(n):
        for (cell, code, L, fx_, fy_) in fan(V, i):
            if owns(i, cell, code):
                where[(i, cell, code)] = len(e_i)
                e_i.append(i)
                e_j.append(np.int32(np.uint32(cell | (code << CODE_SHIFT)).view(np.int32)))
                e_len.append(L)
                e_fx.append(fx_)
                e_fy.append(fy_)
    off, idx = [0], []
    for i in range(n):
        for (cell, code, L, fx_, fy_) in fan(V, i):
            if owns(i, cell, code):
                idx.append(2 * where[(i, cell, code)])
            else:
                back = 0 if code == 0 else 9 - code
                idx.append(2 * where[(cell, i, back)] + 1)
        off.append(len(idx))

    class M:
        pass
    m = M()
    m.n_cells, m.n_edges, m.n_csr = n, len(e_i), len(idx)
    m.px, m.py, m.sx, m.sy, m.area = V.px, V.py, V.sx, V.sy, V.area
    m.e_i = np.array(e_i, dtype=np.int32)
    m.e_j = np.array(e_j, dtype=np.int32)
    m.e_len, m.e_fx, m.e_fy = (np.array(a, dtype=np.float64) for a in (e_len, e_fx, e_fy))
    m.off = np.array(off, dtype=np.int32)
    m.idx = np.array(idx, dtype=np.int32)
    m.box, m.bc = V.box, V.bc
    return m
