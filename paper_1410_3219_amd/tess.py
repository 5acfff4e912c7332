"""ctypes binding of the host input stage (``librichtess.so``, rich_tess.h).

The tessellation (paper section 2.1) turns mesh-generating points into the
flat Voronoi mesh arrays that the device path and the oracle both consume.
This module only marshals arguments; the work is in the C++ library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librichtess.so")

BC_WALLS = 0
BC_PERIODIC = 1
CELL_MASK = 0x0FFFFFFF
CODE_SHIFT = 28
CODE_WALL_X0, CODE_WALL_X1, CODE_WALL_Y0, CODE_WALL_Y1 = 9, 10, 11, 12

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class MeshHostC(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int64), ("n_edges", C.c_int64), ("n_csr", C.c_int64),
        ("px", _dp), ("py", _dp), ("sx", _dp), ("sy", _dp), ("area", _dp),
        ("e_i", _ip), ("e_j", _ip),
        ("e_len", _dp), ("e_fx", _dp), ("e_fy", _dp),
        ("off", _ip), ("idx", _ip), ("eoff", _ip),
        ("box", C.c_double * 4), ("bc", C.c_uint32),
        ("n_ghosts", C.c_int64), ("n_dropped", C.c_int64),
        ("band", C.c_double), ("n_rebuilds", C.c_int32), ("n_exact", C.c_int64),
        ("t_triangulate", C.c_double), ("t_voronoi", C.c_double),
    ]


class TriHostC(C.Structure):
    _fields_ = [
        ("n_pts", C.c_int64), ("n_tri", C.c_int64),
        ("x", _dp), ("y", _dp), ("ghost_src", _ip), ("tri", _ip),
    ]


TESS_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, _dp, _dp, C.c_int64, _dp, C.c_uint32,
                      C.POINTER(MeshHostC))

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        L.rich_tess_build.argtypes = [_dp, _dp, C.c_int64, _dp, C.c_uint32,
                                      C.c_int32, C.POINTER(MeshHostC)]
        L.rich_tess_build.restype = C.c_int
        L.rich_tess_free.argtypes = [C.POINTER(MeshHostC)]
        L.rich_tess_free.restype = None
        L.rich_tess_triangles.argtypes = [_dp, _dp, C.c_int64, _dp, C.c_uint32,
                                          C.POINTER(TriHostC)]
        L.rich_tess_triangles.restype = C.c_int
        L.rich_tess_free_tri.argtypes = [C.POINTER(TriHostC)]
        L.rich_tess_free_tri.restype = None
        L.rich_tess_orient2d.argtypes = [_dp, _dp, _dp]
        L.rich_tess_orient2d.restype = C.c_int
        L.rich_tess_incircle.argtypes = [_dp, _dp, _dp, _dp]
        L.rich_tess_incircle.restype = C.c_int
        L.rich_tess_hilbert_order.argtypes = [_dp, _dp, C.c_int64, _dp,
                                              C.POINTER(C.c_int64)]
        L.rich_tess_hilbert_order.restype = C.c_int
        L.rich_tess_lloyd.argtypes = [_dp, _dp, C.c_int64, _dp, C.c_uint32,
                                      C.c_int32, C.c_int32]
        L.rich_tess_lloyd.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


class TessError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what} failed with status {status}")
        self.status = status


@dataclass
class HostMesh:
    """Flat Voronoi mesh arrays (see rich_mesh_host in rich_tess.h)."""
    px: np.ndarray
    py: np.ndarray
    sx: np.ndarray
    sy: np.ndarray
    area: np.ndarray
    e_i: np.ndarray
    e_j: np.ndarray
    e_len: np.ndarray
    e_fx: np.ndarray
    e_fy: np.ndarray
    off: np.ndarray
    idx: np.ndarray
    eoff: np.ndarray
    box: tuple
    bc: int
    diag: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return int(self.px.shape[0])

    @property
    def n_edges(self):
        return int(self.e_i.shape[0])

    @property
    def n_csr(self):
        return int(self.idx.shape[0])

    def nb_cell(self):
        return (self.e_j.view(np.uint32) & CELL_MASK).astype(np.int64)

    def nb_code(self):
        return (self.e_j.view(np.uint32) >> CODE_SHIFT).astype(np.int64)

    ARRAYS = ("px", "py", "sx", "sy", "area", "e_i", "e_j", "e_len", "e_fx",
              "e_fy", "off", "idx", "eoff")


def _copy(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    ct = C.c_double if dtype == np.float64 else C.c_int32
    buf = C.cast(ptr, C.POINTER(ct * n)).contents
    return np.frombuffer(buf, dtype=dtype).copy()


def mesh_from_c(m: MeshHostC) -> HostMesh:
    n, ne, nc = m.n_cells, m.n_edges, m.n_csr
    f8, i4 = np.float64, np.int32
    return HostMesh(
        px=_copy(m.px, n, f8), py=_copy(m.py, n, f8),
        sx=_copy(m.sx, n, f8), sy=_copy(m.sy, n, f8), area=_copy(m.area, n, f8),
        e_i=_copy(m.e_i, ne, i4), e_j=_copy(m.e_j, ne, i4),
        e_len=_copy(m.e_len, ne, f8), e_fx=_copy(m.e_fx, ne, f8),
        e_fy=_copy(m.e_fy, ne, f8),
        off=_copy(m.off, n + 1, i4), idx=_copy(m.idx, nc, i4),
        eoff=_copy(m.eoff, n + 1, i4),
        box=tuple(m.box), bc=int(m.bc),
        diag=dict(n_ghosts=m.n_ghosts, n_dropped=m.n_dropped, band=m.band,
                  n_rebuilds=m.n_rebuilds, n_exact=m.n_exact,
                  t_triangulate=m.t_triangulate, t_voronoi=m.t_voronoi))


def rich_tess_build(px, py, box, bc, n_threads=0) -> HostMesh:
    """Voronoi mesh of the points (px, py) in box=(x0, y0, x1, y1)."""
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    m = MeshHostC()
    st = lib().rich_tess_build(_d(px), _d(py), px.shape[0], _d(b), bc, n_threads,
                               C.byref(m))
    if st != 0:
        raise TessError(st, "rich_tess_build")
    try:
        return mesh_from_c(m)
    finally:
        lib().rich_tess_free(C.byref(m))


def rich_tess_triangles(px, py, box, bc):
    """Delaunay triangles (real + ghost points) that touch a real point."""
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    t = TriHostC()
    st = lib().rich_tess_triangles(_d(px), _d(py), px.shape[0], _d(b), bc, C.byref(t))
    if st != 0:
        raise TessError(st, "rich_tess_triangles")
    try:
        x = _copy(t.x, t.n_pts, np.float64)
        y = _copy(t.y, t.n_pts, np.float64)
        gs = _copy(t.ghost_src, t.n_pts, np.int32)
        tri = _copy(t.tri, 3 * t.n_tri, np.int32).reshape(-1, 3)
        return x, y, gs, tri
    finally:
        lib().rich_tess_free_tri(C.byref(t))


def rich_tess_orient2d(a, b, c):
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c)]
    return lib().rich_tess_orient2d(*[_d(v) for v in arr])


def rich_tess_incircle(a, b, c, d):
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d)]
    return lib().rich_tess_incircle(*[_d(v) for v in arr])


def rich_tess_hilbert_order(px, py, box):
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    perm = np.zeros(px.shape[0], dtype=np.int64)
    st = lib().rich_tess_hilbert_order(_d(px), _d(py), px.shape[0], _d(b),
                                       perm.ctypes.data_as(C.POINTER(C.c_int64)))
    if st != 0:
        raise TessError(st, "rich_tess_hilbert_order")
    return perm


def rich_tess_lloyd(px, py, box, bc, iters, n_threads=0):
    px = np.array(px, dtype=np.float64, copy=True)
    py = np.array(py, dtype=np.float64, copy=True)
    b = np.ascontiguousarray(box, dtype=np.float64)
    st = lib().rich_tess_lloyd(_d(px), _d(py), px.shape[0], _d(b), bc, iters, n_threads)
    if st != 0:
        raise TessError(st, "rich_tess_lloyd")
    return px, py
