"""ctypes binding of the device path (librich.so, rich.h).

Argument marshalling only: every step of the stage runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  Importing this
module does not need a GPU; calling into the library does, and a missing
library raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librich.so")

RICH_OK, RICH_E_INVAL, RICH_E_NOMEM, RICH_E_DEVICE, RICH_E_DOMAIN, RICH_E_MESH = 0, -1, -2, -3, -4, -5
FLAG_DOMAIN, FLAG_VACUUM = 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


class RichMesh(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int64), ("n_edges", C.c_int64), ("n_csr", C.c_int64),
        ("cells", _vp), ("edges", _vp),
        ("off", _vp), ("idx", _vp), ("eoff", _vp),
        ("box", C.c_double * 4), ("bc", C.c_uint32),
    ]


CELL_BYTES, EDGE_BYTES = 48, 32   # sizeof(rich_cell), sizeof(rich_edge)


class RichMeshBufs(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("cap_edges", C.c_int64), ("cap_csr", C.c_int64),
                ("cells", _vp), ("edges", _vp), ("off", _vp), ("idx", _vp), ("eoff", _vp)]


class RichRetessInfo(C.Structure):
    _fields_ = [("flags", C.c_int32), ("sticky", C.c_int32), ("n_edges", C.c_int64),
                ("n_csr", C.c_int64), ("n_dropped", C.c_int64), ("area_sum", C.c_double),
                ("n_clipped", C.c_int64)]


RETESS_POINT, RETESS_FAN, RETESS_CLIP, RETESS_ASYM, RETESS_AREA, RETESS_CAP = 1, 2, 4, 8, 16, 32


class RichBatchPlan(C.Structure):
    _fields_ = [("n_runs", C.c_int32), ("n_cell_tiles", C.c_int32),
                ("n_flux_tiles", C.c_int32 * 2), ("n_group", C.c_int32 * 2),
                ("grid_cell", C.c_int32), ("grid_flux", C.c_int32 * 2),
                ("flux_tile", C.c_int32), ("courant", C.c_int32), ("serial", C.c_int64),
                ("table_offset", C.c_int64)]


class RichState(C.Structure):
    _fields_ = [("M", _vp), ("Px", _vp), ("Py", _vp), ("E", _vp), ("x", _vp), ("y", _vp),
                ("n_cells", C.c_int64)]


class RichParams(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("cfl", C.c_double), ("theta", C.c_double),
        ("delta_v", C.c_double), ("delta_p", C.c_double), ("chi", C.c_double),
        ("eta", C.c_double), ("riemann", C.c_int32), ("motion", C.c_int32),
        ("limiter", C.c_int32), ("gx", C.c_double), ("gy", C.c_double),
        ("integrator", C.c_int32),
    ]


class HostMeshView(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int64), ("n_edges", C.c_int64), ("n_csr", C.c_int64),
        ("px", _dp), ("py", _dp), ("sx", _dp), ("sy", _dp), ("area", _dp),
        ("e_i", _ip), ("e_j", _ip), ("e_len", _dp), ("e_fx", _dp), ("e_fy", _dp),
        ("off", _ip), ("idx", _ip), ("eoff", _ip),
    ]


TESS_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, _dp, _dp, C.c_int64, _dp, C.c_uint32,
                      C.POINTER(HostMeshView))
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(HostMeshView))


@dataclass
class Params:
    """Scheme parameters (rich_params); defaults are the paper's."""
    gamma: float = 5.0 / 3.0
    cfl: float = 0.3
    theta: float = 0.5
    delta_v: float = 0.2
    delta_p: float = 0.7
    chi: float = 0.15
    eta: float = 0.02
    riemann: int = 0
    motion: int = 1
    limiter: int = 0
    gx: float = 0.0     # uniform external acceleration
    gy: float = 0.0
    integrator: int = 0   # 0 time-centred fluxes (two stages), 1 extrapolated fluxes

    def c(self):
        return RichParams(self.gamma, self.cfl, self.theta, self.delta_v, self.delta_p,
                          self.chi, self.eta, self.riemann, self.motion, self.limiter,
                          self.gx, self.gy, self.integrator)


class RichError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        mp, sp, pp = C.POINTER(RichMesh), C.POINTER(RichState), C.POINTER(RichParams)
        L.rich_params_default.argtypes = [pp, C.c_double]
        L.rich_params_default.restype = None
        L.rich_workspace_size.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
        L.rich_stage.argtypes = [mp, sp, sp, sp, C.c_double, pp, _vp, C.c_size_t, _vp]
        L.rich_stage_noalloc.argtypes = [mp, sp, sp, sp, C.c_double, pp, _vp, _vp]
        L.rich_stage_flags.argtypes = [_vp, _vp, _ip]
        L.rich_stage_debug.argtypes = [mp, sp, sp, sp, C.c_double, pp, _vp, C.c_size_t, _vp, _vp,
                                       _vp]
        L.rich_stage_accel.argtypes = [mp, sp, sp, sp, C.c_double, pp, _vp, _vp, _vp, C.c_size_t,
                                       _vp]
        L.rich_cfl_dt.argtypes = [mp, sp, pp, _dp, _vp, C.c_size_t, _vp]
        L.rich_area_rate.argtypes = [mp, sp, pp, _vp, _vp, C.c_size_t, _vp]
        L.rich_stage_courant.argtypes = [mp, sp, sp, sp, C.c_double, pp, _vp, C.c_size_t, _vp]
        L.rich_stage_dt_of.argtypes = [mp, sp, sp, sp, C.c_double, _vp, pp, _vp, C.c_size_t,
                                       _vp]
        L.rich_stage_dt.argtypes = [_vp, _vp, _dp]
        L.rich_retess_capacity.argtypes = [C.c_int64, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int64)]
        L.rich_retess_workspace_size.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
        L.rich_retess.argtypes = [mp, _vp, _vp, C.POINTER(RichMeshBufs), _vp, C.c_size_t, _vp]
        L.rich_retess_view.argtypes = [C.POINTER(RichMeshBufs), _dp, C.c_uint32, mp]
        L.rich_retess_result.argtypes = [_vp, _vp, C.POINTER(RichRetessInfo)]
        L.rich_retess_batch_workspace_size.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
        L.rich_retess_batch.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                        C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp),
                                        C.POINTER(C.c_size_t), _vp, C.c_size_t, _vp]
        L.rich_retess_batch_result.argtypes = [C.c_int32, _vp, _vp, C.POINTER(RichRetessInfo),
                                               _ip]
        L.rich_retess_batch_flags_async.argtypes = [C.c_int32, _vp, _vp, _vp]
        L.rich_mesh_pack.argtypes = [C.POINTER(HostMeshView), _vp, _vp]
        L.rich_mesh_pack.restype = C.c_int
        L.rich_strerror.argtypes = [C.c_int]
        L.rich_strerror.restype = C.c_char_p
        L.rich_profile_enable.argtypes = [C.c_int]
        L.rich_profile_read.argtypes = [C.c_char_p, _dp, C.POINTER(C.c_int64)]
        for f in ("rich_workspace_size", "rich_stage", "rich_stage_flags", "rich_cfl_dt",
                  "rich_stage_courant", "rich_stage_dt_of", "rich_stage_dt", "rich_area_rate",
                  "rich_retess_capacity", "rich_retess_workspace_size", "rich_retess",
                  "rich_retess_view", "rich_retess_result", "rich_retess_batch_workspace_size",
                  "rich_retess_batch", "rich_retess_batch_result",
                  "rich_retess_batch_flags_async", "rich_profile_enable", "rich_profile_read"):
            getattr(L, f).restype = C.c_int
        if hasattr(L, "rich_stage_batch"):
            L.rich_batch_workspace_size.argtypes = [C.c_int32, C.POINTER(C.c_int64),
                                                    C.POINTER(C.c_size_t)]
            # arrays of struct addresses (const T* const*), passed as void**
            L.rich_stage_batch.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                           C.POINTER(_vp), C.POINTER(_vp), _dp, C.POINTER(_vp),
                                           _vp, C.c_size_t, _vp]
            L.rich_stage_batch_accel.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                                 C.POINTER(_vp), C.POINTER(_vp), _dp,
                                                 C.POINTER(_vp), C.POINTER(_vp),
                                                 C.POINTER(_vp), _vp, C.c_size_t, _vp]
            L.rich_batch_flags.argtypes = [C.c_int32, _vp, _vp, _ip]
            L.rich_batch_flags_async.argtypes = [C.c_int32, _vp, _vp, _vp]
            L.rich_stage_batch_prepare.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                                   C.POINTER(_vp), C.POINTER(_vp), _dp,
                                                   C.POINTER(_vp), _vp, C.c_size_t, _vp,
                                                   C.POINTER(RichBatchPlan)]
            L.rich_stage_batch_launch.argtypes = [C.POINTER(RichBatchPlan), _vp, _vp]
            L.rich_stage_batch_prepare_tile.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                                        C.POINTER(_vp), C.POINTER(_vp), _dp,
                                                        C.POINTER(_vp), C.c_int32, _vp,
                                                        C.c_size_t, _vp, C.POINTER(RichBatchPlan)]
            L.rich_stage_batch_prepare_courant.argtypes = [
                C.c_int32, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), _dp,
                C.POINTER(_vp), C.c_int32, _vp, _vp, C.c_size_t, _vp, C.POINTER(RichBatchPlan)]
            L.rich_batch_dt.argtypes = [C.c_int32, _vp, _vp, _dp]
            L.rich_stage_batch_autotune.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                                    C.POINTER(_vp), C.POINTER(_vp), _dp,
                                                    C.POINTER(_vp), C.c_int32, _vp, C.c_size_t,
                                                    _vp, _ip, _dp]
            for f in ("rich_batch_workspace_size", "rich_stage_batch", "rich_batch_flags",
                      "rich_batch_flags_async", "rich_stage_batch_prepare",
                      "rich_stage_batch_launch", "rich_stage_batch_prepare_tile",
                      "rich_stage_batch_autotune", "rich_stage_batch_prepare_courant",
                      "rich_batch_dt"):
                getattr(L, f).restype = C.c_int
        if hasattr(L, "rich_step"):
            L.rich_ctx_create.argtypes = [C.POINTER(_vp)]
            L.rich_ctx_destroy.argtypes = [_vp]
            L.rich_ctx_destroy.restype = None
            L.rich_ctx_set_mesh.argtypes = [_vp, C.POINTER(HostMeshView), _dp, C.c_uint32, _vp]
            L.rich_ctx_mesh.argtypes = [_vp, mp]
            L.rich_ctx_set_device_tess.argtypes = [_vp, C.c_int32]
            L.rich_ctx_tess_counts.argtypes = [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
            L.rich_step.argtypes = [_vp, sp, C.c_double, pp, _vp, _vp, _vp, _vp]
            L.rich_step_accel.argtypes = [_vp, sp, C.c_double, pp, _vp, _vp, _vp, _vp, _vp, _vp]
            L.rich_step_batch.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp), _dp,
                                          C.POINTER(_vp), _vp, _vp, C.POINTER(_vp), C.c_int32,
                                          _ip, _vp, C.c_size_t, _vp]
            L.rich_step_batch_accel.argtypes = [C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                                _dp, C.POINTER(_vp), C.POINTER(_vp),
                                                C.POINTER(_vp), _vp, _vp, C.POINTER(_vp),
                                                C.c_int32, _ip, _vp, C.c_size_t, _vp]
            for f in ("rich_ctx_create", "rich_ctx_set_mesh", "rich_ctx_mesh", "rich_step",
                      "rich_step_batch", "rich_step_batch_accel", "rich_ctx_set_device_tess", "rich_ctx_tess_counts"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def strerror(status):
    try:
        return lib().rich_strerror(int(status)).decode()
    except Exception:
        return "unknown"


def _check(st, what):
    if st != RICH_OK:
        raise RichError(st, what)


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dense(t, stream):
    """t itself when contiguous, else a contiguous copy that is safe to hand
    to work enqueued on `stream`: the copy is made on torch's current stream,
    so `stream` first waits for it, and the allocator is told the copy is in
    use there (it is not reused before that stream's work completes)."""
    if t.is_contiguous():
        return t
    import torch
    c = t.contiguous()
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())
        c.record_stream(stream)
    return c


def _accel_field(a, n, device, name, contiguous=False):
    """Check a per-cell acceleration field before its pointer is taken: a
    (2, n) float64 tensor on the state's GPU (a host tensor's pointer, or
    another dtype's bits read as doubles, would reach the kernels)."""
    import torch
    if not isinstance(a, torch.Tensor):
        raise RichError(RICH_E_INVAL, f"{name}: the field must be a torch tensor")
    if a.dtype != torch.float64:
        raise RichError(RICH_E_INVAL, f"{name}: the field must be float64, not {a.dtype}")
    if a.device.type != "cuda" or a.device != device:
        raise RichError(RICH_E_INVAL,
                        f"{name}: the field must be on the state's device {device}, not {a.device}")
    if tuple(a.shape) != (2, n):
        raise RichError(RICH_E_INVAL, f"{name}: the field must be (2, {n}), not {tuple(a.shape)}")
    if contiguous and not a.is_contiguous():
        raise RichError(RICH_E_INVAL, f"{name}: the field must be contiguous")


# ---------------------------------------------------------------------------
# device-resident mesh and state (torch tensors)
# ---------------------------------------------------------------------------
@dataclass
class DeviceMesh:
    t: dict
    n_cells: int
    n_edges: int
    n_csr: int
    box: tuple
    bc: int
    _c: RichMesh = field(default=None, repr=False)

    @classmethod
    def from_host(cls, hm, device="cuda"):
        """Pack the host stage's arrays into the device records (rich_mesh_pack)
        and upload them with the CSR arrays."""
        import torch
        cells, edges = pack_mesh(hm)
        t = {"cells": torch.from_numpy(cells).to(device),
             "edges": torch.from_numpy(edges).to(device)}
        for k in ("off", "idx", "eoff"):
            t[k] = torch.from_numpy(np.ascontiguousarray(getattr(hm, k))).to(device)
        return cls(t, hm.n_cells, hm.n_edges, hm.n_csr, tuple(hm.box), int(hm.bc))

    def c(self):
        if self._c is None:
            p = {k: C.c_void_p(v.data_ptr()) for k, v in self.t.items()}
            self._c = RichMesh(self.n_cells, self.n_edges, self.n_csr,
                               p["cells"], p["edges"], p["off"], p["idx"], p["eoff"],
                               (C.c_double * 4)(*self.box), self.bc)
        return self._c

    def nbytes(self):
        return sum(v.numel() * v.element_size() for v in self.t.values())


@dataclass
class DeviceState:
    """Q (4, n): M, Px, Py, E extensive totals; X (2, n): points."""
    Q: "torch.Tensor"
    X: "torch.Tensor"
    _c: RichState = field(default=None, repr=False, compare=False)

    @classmethod
    def from_host(cls, Q, X, device="cuda"):
        import torch
        return cls(torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(device))

    @classmethod
    def empty_like(cls, other):
        import torch
        return cls(torch.empty_like(other.Q), torch.empty_like(other.X))

    @property
    def n(self):
        return int(self.Q.shape[1])

    def __setattr__(self, name, value):
        if name in ("Q", "X"):
            object.__setattr__(self, "_c", None)   # a new tensor: rebuild the view
        object.__setattr__(self, name, value)

    def c(self):
        """The C view (rows of Q and X are contiguous), built once per pair
        of tensors (in-place updates keep the storage)."""
        if self._c is None:
            q, x = self.Q, self.X
            assert q.is_contiguous() and x.is_contiguous()
            assert q.dtype == x.dtype and q.element_size() == 8
            n = int(q.shape[1])
            qb, xb = q.data_ptr(), x.data_ptr()
            object.__setattr__(self, "_c", RichState(qb, qb + 8 * n, qb + 16 * n, qb + 24 * n,
                                                     xb, xb + 8 * n, n))
        return self._c

    def numpy(self):
        return self.Q.cpu().numpy(), self.X.cpu().numpy()


def rich_workspace_size(n_cells):
    b = C.c_size_t(0)
    _check(lib().rich_workspace_size(int(n_cells), C.byref(b)), "rich_workspace_size")
    return int(b.value)


def workspace(n_cells, device="cuda"):
    import torch
    nb = rich_workspace_size(n_cells)
    return torch.empty(nb, dtype=torch.uint8, device=device)


def rich_stage(mesh: DeviceMesh, src: DeviceState, base: DeviceState, out: DeviceState, h,
               params: Params, ws, stream=None):
    """Enqueue one stage; returns immediately (see rich_stage_flags)."""
    st = lib().rich_stage(C.byref(mesh.c()), C.byref(src.c()), C.byref(base.c()),
                          C.byref(out.c()), float(h), C.byref(params.c()),
                          C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
    _check(st, "rich_stage")


NOALLOC_MAX_CELLS = 1048576   # RICH_NOALLOC_MAX_CELLS


def rich_stage_noalloc(mesh: DeviceMesh, src: DeviceState, base: DeviceState, out: DeviceState,
                       h, params: Params, flag_out=None, stream=None):
    """Enqueue one stage on the library's own scratch (no workspace; at most
    NOALLOC_MAX_CELLS cells; calls on one GPU must not overlap).  flag_out: an
    int32 device tensor of one element that receives the stage's flag word,
    or None."""
    fp = None
    if flag_out is not None:
        import torch
        if flag_out.dtype != torch.int32 or flag_out.numel() < 1 or flag_out.device.type != "cuda":
            raise RichError(RICH_E_INVAL, "rich_stage_noalloc: flag_out must be an int32 device tensor")
        fp = C.c_void_p(flag_out.data_ptr())
    st = lib().rich_stage_noalloc(C.byref(mesh.c()), C.byref(src.c()), C.byref(base.c()),
                                  C.byref(out.c()), float(h), C.byref(params.c()), fp,
                                  _stream_ptr(stream))
    _check(st, "rich_stage_noalloc")


def rich_stage_accel(mesh: DeviceMesh, src: DeviceState, base: DeviceState, out: DeviceState,
                     h, params: Params, accel, ws, stream=None):
    """Enqueue one stage with a per-cell acceleration accel (2, n), a float64
    device tensor, added to the uniform one of params."""
    n = mesh.n_cells
    _accel_field(accel, n, base.Q.device, "rich_stage_accel")
    a = _dense(accel, stream)
    st = lib().rich_stage_accel(C.byref(mesh.c()), C.byref(src.c()), C.byref(base.c()),
                                C.byref(out.c()), float(h), C.byref(params.c()),
                                C.c_void_p(a.data_ptr()), C.c_void_p(a.data_ptr() + 8 * n),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
    _check(st, "rich_stage_accel")


def rich_stage_debug(mesh: DeviceMesh, src: DeviceState, base: DeviceState, out: DeviceState,
                     h, params: Params, ws, stream=None):
    """rich_stage plus the branch records; returns (cell_bits, edge_bits),
    uint8 device tensors (bit meanings in rich.h)."""
    import torch
    dev = src.Q.device
    cb = torch.zeros(mesh.n_cells, dtype=torch.uint8, device=dev)
    eb = torch.zeros(max(mesh.n_edges, 1), dtype=torch.uint8, device=dev)
    st = lib().rich_stage_debug(C.byref(mesh.c()), C.byref(src.c()), C.byref(base.c()),
                                C.byref(out.c()), float(h), C.byref(params.c()),
                                C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(cb.data_ptr()),
                                C.c_void_p(eb.data_ptr()), _stream_ptr(stream))
    _check(st, "rich_stage_debug")
    return cb, eb[:mesh.n_edges]


def rich_stage_flags(ws, stream=None):
    f = C.c_int32(0)
    _check(lib().rich_stage_flags(C.c_void_p(ws.data_ptr()), _stream_ptr(stream), C.byref(f)),
           "rich_stage_flags")
    return int(f.value)


def rich_cfl_dt(mesh: DeviceMesh, state: DeviceState, params: Params, ws, stream=None):
    dt = C.c_double(0.0)
    st = lib().rich_cfl_dt(C.byref(mesh.c()), C.byref(state.c()), C.byref(params.c()),
                           C.byref(dt), C.c_void_p(ws.data_ptr()), ws.numel(),
                           _stream_ptr(stream))
    _check(st, "rich_cfl_dt")
    return dt.value


def rich_area_rate(mesh: DeviceMesh, state: DeviceState, params: Params, ws, stream=None):
    """dA/dt of every cell implied by the moving edges (device tensor)."""
    import torch
    adot = torch.empty(mesh.n_cells, dtype=torch.float64, device=state.Q.device)
    st = lib().rich_area_rate(C.byref(mesh.c()), C.byref(state.c()), C.byref(params.c()),
                              C.c_void_p(adot.data_ptr()), C.c_void_p(ws.data_ptr()),
                              ws.numel(), _stream_ptr(stream))
    _check(st, "rich_area_rate")
    return adot


def rich_stage_courant(mesh: DeviceMesh, src: DeviceState, base: DeviceState,
                       out: DeviceState, h_factor, params: Params, ws, stream=None):
    """Enqueue a stage whose step is h_factor * the Courant dt of src, both
    taken on the device (dt stays in ws; see rich_stage_dt)."""
    st = lib().rich_stage_courant(C.byref(mesh.c()), C.byref(src.c()), C.byref(base.c()),
                                  C.byref(out.c()), float(h_factor), C.byref(params.c()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
    _check(st, "rich_stage_courant")


def rich_stage_dt_of(mesh: DeviceMesh, src: DeviceState, base: DeviceState, out: DeviceState,
                     h_factor, dt_ws, params: Params, ws, stream=None):
    """Enqueue a stage whose step is h_factor * the dt held in workspace dt_ws."""
    st = lib().rich_stage_dt_of(C.byref(mesh.c()), C.byref(src.c()), C.byref(base.c()),
                                C.byref(out.c()), float(h_factor),
                                C.c_void_p(dt_ws.data_ptr()), C.byref(params.c()),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
    _check(st, "rich_stage_dt_of")


def rich_stage_dt(ws, stream=None):
    """Synchronise and return the dt the last rich_stage_courant on ws wrote."""
    dt = C.c_double(0.0)
    _check(lib().rich_stage_dt(C.c_void_p(ws.data_ptr()), _stream_ptr(stream), C.byref(dt)),
           "rich_stage_dt")
    return dt.value


# ---------------------------------------------------------------------------
# device re-tessellation
# ---------------------------------------------------------------------------
def rich_retess_capacity(n_cells):
    ce, cc = C.c_int64(0), C.c_int64(0)
    _check(lib().rich_retess_capacity(int(n_cells), C.byref(ce), C.byref(cc)),
           "rich_retess_capacity")
    return int(ce.value), int(cc.value)


def rich_retess_workspace_size(n_cells):
    b = C.c_size_t(0)
    _check(lib().rich_retess_workspace_size(int(n_cells), C.byref(b)),
           "rich_retess_workspace_size")
    return int(b.value)


def retess_workspace(n_cells, device="cuda"):
    """Workspace of rich_retess, zeroed (its result header starts cleared)."""
    import torch
    return torch.zeros(rich_retess_workspace_size(n_cells), dtype=torch.uint8, device=device)


class DeviceMeshBufs:
    """Output buffers of rich_retess for n_cells cells, at full capacity."""

    def __init__(self, n_cells, box, bc, device="cuda"):
        import torch
        ce, cc = rich_retess_capacity(n_cells)
        self.n_cells, self.cap_edges, self.cap_csr = int(n_cells), ce, cc
        self.box, self.bc = tuple(float(v) for v in box), int(bc)
        u8, i32 = torch.uint8, torch.int32
        self.t = {"cells": torch.empty(CELL_BYTES * n_cells, dtype=u8, device=device),
                  "edges": torch.empty(EDGE_BYTES * ce, dtype=u8, device=device),
                  "off": torch.zeros(n_cells + 1, dtype=i32, device=device),
                  "idx": torch.zeros(cc, dtype=i32, device=device),
                  "eoff": torch.zeros(n_cells + 1, dtype=i32, device=device)}
        p = {k: C.c_void_p(v.data_ptr()) for k, v in self.t.items()}
        self._c = RichMeshBufs(self.n_cells, ce, cc, p["cells"], p["edges"], p["off"],
                               p["idx"], p["eoff"])

    def c(self):
        return self._c

    def mesh(self):
        """The stage's view (edge and CSR counts are the capacities)."""
        return DeviceMesh(self.t, self.n_cells, self.cap_edges, self.cap_csr, self.box,
                          self.bc)


def rich_retess(prev: DeviceMesh, X, bufs: DeviceMeshBufs, ws, stream=None):
    """Enqueue the re-tessellation of points X (2, n) (device) with candidates
    from `prev` into `bufs`; read the outcome with rich_retess_result."""
    X = _dense(X, stream)
    n = prev.n_cells
    xp = C.c_void_p(X.data_ptr())
    yp = C.c_void_p(X.data_ptr() + 8 * n)
    st = lib().rich_retess(C.byref(prev.c()), xp, yp, C.byref(bufs.c()),
                           C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
    _check(st, "rich_retess")


def rich_retess_result(ws, stream=None):
    """(status, info): status RICH_E_MESH when the last call failed."""
    info = RichRetessInfo()
    st = lib().rich_retess_result(C.c_void_p(ws.data_ptr()), _stream_ptr(stream),
                                  C.byref(info))
    if st not in (RICH_OK, RICH_E_MESH):
        _check(st, "rich_retess_result")
    return st, {"flags": info.flags, "sticky": info.sticky, "n_edges": info.n_edges,
                "n_csr": info.n_csr, "n_dropped": info.n_dropped, "area_sum": info.area_sum,
                "n_clipped": info.n_clipped}


def rich_retess_batch(prevs, Xs, bufs, wss, bws=None, stream=None):
    """Re-tessellate several runs in one launch per kernel; returns the batch
    workspace to pass to rich_retess_batch_result."""
    import torch
    n = len(prevs)
    if bws is None:
        b = C.c_size_t(0)
        _check(lib().rich_retess_batch_workspace_size(n, C.byref(b)),
               "rich_retess_batch_workspace_size")
        bws = torch.empty(int(b.value), dtype=torch.uint8, device=Xs[0].device)
    Xs = [_dense(X, stream) for X in Xs]
    ad = C.addressof
    pm = (_vp * n)(*[ad(m.c()) for m in prevs])
    xp = (_vp * n)(*[X.data_ptr() for X in Xs])
    yp = (_vp * n)(*[X.data_ptr() + 8 * m.n_cells for X, m in zip(Xs, prevs)])
    op = (_vp * n)(*[ad(b_.c()) for b_ in bufs])
    wp = (_vp * n)(*[w.data_ptr() for w in wss])
    wb = (C.c_size_t * n)(*[w.numel() for w in wss])
    _check(lib().rich_retess_batch(n, pm, xp, yp, op, wp, wb, C.c_void_p(bws.data_ptr()),
                                   bws.numel(), _stream_ptr(stream)), "rich_retess_batch")
    return bws


def rich_retess_batch_result(n, bws, stream=None):
    """[(status, info dict)] of the runs of the last rich_retess_batch on bws."""
    info = (RichRetessInfo * n)()
    st = (C.c_int32 * n)()
    _check(lib().rich_retess_batch_result(n, C.c_void_p(bws.data_ptr()), _stream_ptr(stream),
                                          info, st), "rich_retess_batch_result")
    return [(int(st[r]), {"flags": info[r].flags, "sticky": info[r].sticky,
                          "n_edges": info[r].n_edges, "n_csr": info[r].n_csr,
                          "n_dropped": info[r].n_dropped, "area_sum": info[r].area_sum,
                          "n_clipped": info[r].n_clipped})
            for r in range(n)]


def rich_retess_batch_flags_async(n, bws, host_flags, stream=None):
    """Enqueue the copy of the n runs' RICH_RETESS_* flags of the last
    rich_retess_batch on bws into host_flags (a pinned int32 CPU tensor of at
    least n elements); valid once the stream passes it (nonzero: the run's
    mesh was not built)."""
    import torch
    if host_flags.dtype != torch.int32 or host_flags.numel() < n or host_flags.is_cuda:
        raise RichError(RICH_E_INVAL, "rich_retess_batch_flags_async: host_flags must be an "
                                      f"int32 CPU tensor of at least {n} elements")
    _check(lib().rich_retess_batch_flags_async(n, C.c_void_p(bws.data_ptr()),
                                               _stream_ptr(stream),
                                               C.c_void_p(host_flags.data_ptr())),
           "rich_retess_batch_flags_async")


def mesh_to_host(dm: DeviceMesh, n_edges=None, n_csr=None):
    """Device mesh records back as host-stage arrays (for checks)."""
    cells = dm.t["cells"].cpu().numpy().view(np.float64).reshape(-1, 6)
    ne = dm.n_edges if n_edges is None else n_edges
    nc = dm.n_csr if n_csr is None else n_csr
    er = dm.t["edges"][:EDGE_BYTES * ne].cpu().numpy()
    ed = er.view(np.dtype([("fx", "<f8"), ("fy", "<f8"), ("len", "<f8"), ("i", "<i4"),
                           ("j", "<i4")]))

    class H:
        pass
    h = H()
    h.n_cells, h.n_edges, h.n_csr = dm.n_cells, ne, nc
    h.px, h.py, h.area, h.sx, h.sy = (np.ascontiguousarray(cells[:, k]) for k in range(5))
    h.e_fx, h.e_fy, h.e_len = (np.ascontiguousarray(ed[k]) for k in ("fx", "fy", "len"))
    h.e_i, h.e_j = np.ascontiguousarray(ed["i"]), np.ascontiguousarray(ed["j"])
    h.off = dm.t["off"].cpu().numpy()
    h.idx = dm.t["idx"][:nc].cpu().numpy()
    h.eoff = dm.t["eoff"].cpu().numpy()
    h.box, h.bc = dm.box, dm.bc
    return h


def rich_profile_enable(on=True):
    _check(lib().rich_profile_enable(1 if on else 0), "rich_profile_enable")


def rich_profile_read(kernel):
    """(total milliseconds, launches) of `kernel` since the last read."""
    ms, n = C.c_double(0.0), C.c_int64(0)
    _check(lib().rich_profile_read(kernel.encode(), C.byref(ms), C.byref(n)),
           "rich_profile_read")
    return ms.value, n.value


# ---------------------------------------------------------------------------
# batched stage
# ---------------------------------------------------------------------------
def rich_batch_workspace_size(n_cells):
    arr = (C.c_int64 * len(n_cells))(*[int(x) for x in n_cells])
    b = C.c_size_t(0)
    _check(lib().rich_batch_workspace_size(len(n_cells), arr, C.byref(b)),
           "rich_batch_workspace_size")
    return int(b.value)


def batch_workspace(n_cells, device="cuda"):
    import torch
    return torch.empty(rich_batch_workspace_size(n_cells), dtype=torch.uint8, device=device)


def _batch_args(meshes, srcs, bases, outs, hs, params):
    n = len(meshes)
    ad = C.addressof
    # the structs stay referenced by the objects that cache them for the call
    mp = (_vp * n)(*[ad(m.c()) for m in meshes])
    spp = (_vp * n)(*[ad(x.c()) for x in srcs])
    bpp = (_vp * n)(*[ad(x.c()) for x in bases])
    opp = (_vp * n)(*[ad(x.c()) for x in outs])
    hh = (C.c_double * n)(*[float(h) for h in hs])
    pc = [p.c() for p in params]
    ppp = (_vp * n)(*[ad(x) for x in pc])
    return n, mp, spp, bpp, opp, hh, ppp, pc


def rich_stage_batch(meshes, srcs, bases, outs, hs, params, ws, stream=None):
    """One stage of len(meshes) independent runs, one launch per kernel phase."""
    n, mp, spp, bpp, opp, hh, ppp, _pc = _batch_args(meshes, srcs, bases, outs, hs, params)
    st = lib().rich_stage_batch(n, mp, spp, bpp, opp, hh, ppp, C.c_void_p(ws.data_ptr()),
                                ws.numel(), _stream_ptr(stream))
    _check(st, "rich_stage_batch")


def rich_stage_batch_accel(meshes, srcs, bases, outs, hs, params, accels, ws, stream=None):
    """rich_stage_batch with per-run per-cell accelerations: accels[r] is a
    contiguous (2, n_r) float64 device tensor, or None for a run without one."""
    n = len(meshes)
    if len(accels) != n:
        raise RichError(RICH_E_INVAL, "rich_stage_batch_accel: one field (or None) per run")
    ax, ay = (_vp * n)(), (_vp * n)()
    for r, a in enumerate(accels):
        if a is None:
            continue
        nc = meshes[r].n_cells
        _accel_field(a, nc, bases[r].Q.device, "rich_stage_batch_accel", contiguous=True)
        ax[r], ay[r] = a.data_ptr(), a.data_ptr() + 8 * nc
    n, mp, spp, bpp, opp, hh, ppp, _pc = _batch_args(meshes, srcs, bases, outs, hs, params)
    st = lib().rich_stage_batch_accel(n, mp, spp, bpp, opp, hh, ppp, ax, ay,
                                      C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
    _check(st, "rich_stage_batch_accel")


def rich_stage_batch_prepare(meshes, srcs, bases, outs, hs, params, ws, stream=None):
    """Upload the descriptors of a batched stage into ws; returns the plan
    that rich_stage_batch_launch replays (the buffers named here must stay
    alive while the plan is used)."""
    n, mp, spp, bpp, opp, hh, ppp, _pc = _batch_args(meshes, srcs, bases, outs, hs, params)
    plan = RichBatchPlan()
    st = lib().rich_stage_batch_prepare(n, mp, spp, bpp, opp, hh, ppp,
                                        C.c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream_ptr(stream), C.byref(plan))
    _check(st, "rich_stage_batch_prepare")
    return plan


def rich_stage_batch_prepare_tile(meshes, srcs, bases, outs, hs, params, tile, ws,
                                  stream=None):
    """rich_stage_batch_prepare with flux tiles of `tile` cells (128, 256, 512)."""
    n, mp, spp, bpp, opp, hh, ppp, _pc = _batch_args(meshes, srcs, bases, outs, hs, params)
    plan = RichBatchPlan()
    st = lib().rich_stage_batch_prepare_tile(n, mp, spp, bpp, opp, hh, ppp, int(tile),
                                             C.c_void_p(ws.data_ptr()), ws.numel(),
                                             _stream_ptr(stream), C.byref(plan))
    _check(st, "rich_stage_batch_prepare_tile")
    return plan


def rich_stage_batch_prepare_courant(meshes, srcs, bases, outs, factors, params, ws,
                                     dt_ws=None, tile=256, stream=None):
    """A batched stage with each run's step taken on the device (Courant
    condition, section 2.3): with dt_ws None the stage computes every run's
    step from srcs and applies factors[r] times it; otherwise it applies
    factors[r] times the step an earlier Courant stage left in the batch
    workspace dt_ws (which may be ws).  Returns the plan for
    rich_stage_batch_launch."""
    n, mp, spp, bpp, opp, hh, ppp, _pc = _batch_args(meshes, srcs, bases, outs, factors, params)
    plan = RichBatchPlan()
    dtp = None if dt_ws is None else C.c_void_p(dt_ws.data_ptr())
    st = lib().rich_stage_batch_prepare_courant(n, mp, spp, bpp, opp, hh, ppp, int(tile), dtp,
                                                C.c_void_p(ws.data_ptr()), ws.numel(),
                                                _stream_ptr(stream), C.byref(plan))
    _check(st, "rich_stage_batch_prepare_courant")
    return plan


def rich_batch_dt(n, ws, stream=None):
    """The n per-run steps the last Courant stage on the batch workspace ws
    computed (synchronises the stream)."""
    d = (C.c_double * n)()
    _check(lib().rich_batch_dt(n, C.c_void_p(ws.data_ptr()), _stream_ptr(stream), d),
           "rich_batch_dt")
    return list(d)


def rich_stage_batch_autotune(meshes, srcs, bases, outs, hs, params, ws, reps=3, stream=None):
    """(best tile, {tile: ms per launch}) of a batched stage on these runs."""
    n, mp, spp, bpp, opp, hh, ppp, _pc = _batch_args(meshes, srcs, bases, outs, hs, params)
    best = C.c_int32(0)
    ms = (C.c_double * 3)()
    st = lib().rich_stage_batch_autotune(n, mp, spp, bpp, opp, hh, ppp, int(reps),
                                         C.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream_ptr(stream), C.byref(best), ms)
    _check(st, "rich_stage_batch_autotune")
    return int(best.value), {128: ms[0], 256: ms[1], 512: ms[2]}


def rich_stage_batch_launch(plan, ws, stream=None):
    """Enqueue the kernels of a prepared batched stage (capturable)."""
    _check(lib().rich_stage_batch_launch(C.byref(plan), C.c_void_p(ws.data_ptr()),
                                         _stream_ptr(stream)), "rich_stage_batch_launch")


def rich_batch_flags(n, ws, stream=None):
    f = (C.c_int32 * n)()
    _check(lib().rich_batch_flags(n, C.c_void_p(ws.data_ptr()), _stream_ptr(stream), f),
           "rich_batch_flags")
    return list(f)


def rich_batch_flags_async(n, ws, host_flags, stream=None):
    """Enqueue the copy of the n flag words into host_flags (a pinned int32
    CPU tensor of at least n elements); valid once the stream passes it."""
    assert host_flags.dtype.itemsize == 4 and host_flags.numel() >= n
    _check(lib().rich_batch_flags_async(n, C.c_void_p(ws.data_ptr()), _stream_ptr(stream),
                                        C.c_void_p(host_flags.data_ptr())),
           "rich_batch_flags_async")


# ---------------------------------------------------------------------------
# time-centred step driver
# ---------------------------------------------------------------------------
def pack_mesh(hm):
    """Host mesh -> (cells, edges) byte arrays in the device record layout."""
    v, keep = _host_view(hm)
    cells = np.empty(CELL_BYTES * hm.n_cells, dtype=np.uint8)
    edges = np.empty(EDGE_BYTES * max(hm.n_edges, 1), dtype=np.uint8)
    _check(lib().rich_mesh_pack(C.byref(v), cells.ctypes.data_as(_vp),
                                edges.ctypes.data_as(_vp)), "rich_mesh_pack")
    del keep
    return cells, edges[:EDGE_BYTES * hm.n_edges]


def _host_view(hm):
    keep = {k: np.ascontiguousarray(getattr(hm, k)) for k in hm.ARRAYS}
    dp = lambda a: a.ctypes.data_as(_dp)   # noqa: E731
    ip = lambda a: a.ctypes.data_as(_ip)   # noqa: E731
    v = HostMeshView(hm.n_cells, hm.n_edges, hm.n_csr,
                     dp(keep["px"]), dp(keep["py"]), dp(keep["sx"]), dp(keep["sy"]),
                     dp(keep["area"]), ip(keep["e_i"]), ip(keep["e_j"]), dp(keep["e_len"]),
                     dp(keep["e_fx"]), dp(keep["e_fy"]), ip(keep["off"]), ip(keep["idx"]),
                     ip(keep["eoff"]))
    return v, keep


class CtxMesh:
    """Device view of a step driver's current mesh (borrowed)."""

    def __init__(self, cm: RichMesh):
        self._c = cm
        self.n_cells, self.n_edges, self.n_csr = cm.n_cells, cm.n_edges, cm.n_csr

    def c(self):
        return self._c


class RichCtx:
    """rich_ctx: device buffers of one run's time-centred step driver.  The
    host tessellation stage is called through its C adapter, with no Python
    in between."""

    def __init__(self, n_threads=0, device_tess=False):
        from . import tess
        self.h = C.c_void_p()
        _check(lib().rich_ctx_create(C.byref(self.h)), "rich_ctx_create")
        if device_tess:
            _check(lib().rich_ctx_set_device_tess(self.h, 1), "rich_ctx_set_device_tess")
        TL = tess.lib()
        TL.rich_tess_ctx_create.argtypes = [C.c_int32]
        TL.rich_tess_ctx_create.restype = C.c_void_p
        TL.rich_tess_ctx_destroy.argtypes = [C.c_void_p]
        TL.rich_tess_ctx_destroy.restype = None
        self._tl = TL
        self.tess_user = C.c_void_p(TL.rich_tess_ctx_create(int(n_threads)))
        self.tess_fn = C.cast(TL.rich_tess_callback, C.c_void_p)
        self.release_fn = C.cast(TL.rich_tess_release, C.c_void_p)

    def close(self):
        if self.h:
            lib().rich_ctx_destroy(self.h)
            self.h = C.c_void_p()
        if self.tess_user:
            self._tl.rich_tess_ctx_destroy(self.tess_user)
            self.tess_user = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tess_counts(self):
        """(meshes built on the device, meshes the host stage built instead)."""
        d, f = C.c_int64(0), C.c_int64(0)
        _check(lib().rich_ctx_tess_counts(self.h, C.byref(d), C.byref(f)),
               "rich_ctx_tess_counts")
        return int(d.value), int(f.value)

    def set_mesh(self, hm, stream=None):
        v, keep = _host_view(hm)
        box = (C.c_double * 4)(*hm.box)
        _check(lib().rich_ctx_set_mesh(self.h, C.byref(v), box, int(hm.bc),
                                       _stream_ptr(stream)), "rich_ctx_set_mesh")
        del keep

    def mesh(self):
        cm = RichMesh()
        _check(lib().rich_ctx_mesh(self.h, C.byref(cm)), "rich_ctx_mesh")
        return CtxMesh(cm)

    def step(self, state: DeviceState, dt, params: Params, stream=None, accel=None):
        """One time-centred step (rich_step); accel (2, n), a float64 device
        tensor, adds a per-cell acceleration (rich_step_accel)."""
        if accel is None:
            st = lib().rich_step(self.h, C.byref(state.c()), float(dt), C.byref(params.c()),
                                 self.tess_fn, self.release_fn, self.tess_user,
                                 _stream_ptr(stream))
            _check(st, "rich_step")
            return
        n = state.n
        _accel_field(accel, n, state.Q.device, "rich_step_accel")
        a = _dense(accel, stream)
        st = lib().rich_step_accel(self.h, C.byref(state.c()), float(dt), C.byref(params.c()),
                                   C.c_void_p(a.data_ptr()), C.c_void_p(a.data_ptr() + 8 * n),
                                   self.tess_fn, self.release_fn, self.tess_user,
                                   _stream_ptr(stream))
        _check(st, "rich_step_accel")


def rich_step_batch(ctxs, states, dts, params, ws, n_threads=0, stream=None, accels=None):
    """Time-centred step of len(ctxs) runs (RichCtx each) with batched stage
    launches; returns the per-run status list (0: committed).  Raises only
    when the call as a whole failed.  accels: None, or one contiguous (2, n_r)
    float64 device tensor (or None) per run, a per-cell acceleration applied
    in every stage of that run."""
    n = len(ctxs)
    if accels is not None:
        if len(accels) != n:
            raise RichError(RICH_E_INVAL, "rich_step_batch: one field (or None) per run")
        ax, ay = (_vp * n)(), (_vp * n)()
        for r, a in enumerate(accels):
            if a is None:
                continue
            nc = states[r].Q.shape[1]
            _accel_field(a, nc, states[r].Q.device, "rich_step_batch", contiguous=True)
            ax[r], ay[r] = a.data_ptr(), a.data_ptr() + 8 * nc
    ad = C.addressof
    cp = (_vp * n)(*[c.h.value for c in ctxs])
    spp = (_vp * n)(*[ad(s.c()) for s in states])
    dd = (C.c_double * n)(*[float(x) for x in dts])
    pc = [p.c() for p in params]
    ppp = (_vp * n)(*[ad(x) for x in pc])
    users = (_vp * n)(*[c.tess_user.value for c in ctxs])
    status = (C.c_int32 * n)()
    t0 = ctxs[0]
    nt = int(n_threads) if n_threads > 0 else (os.cpu_count() or 1)
    if accels is None:
        rc = lib().rich_step_batch(n, cp, spp, dd, ppp, t0.tess_fn, t0.release_fn, users, nt,
                                   status, C.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream_ptr(stream))
    else:
        rc = lib().rich_step_batch_accel(n, cp, spp, dd, ppp, ax, ay, t0.tess_fn,
                                         t0.release_fn, users, nt, status,
                                         C.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream_ptr(stream))
    st = list(status)
    if rc != RICH_OK and not any(st):   # rejected before any run was looked at
        _check(rc, "rich_step_batch")
    return st   # st[r] == 0: run r was committed
