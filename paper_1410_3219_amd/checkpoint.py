"""Checkpoint and resume of a run: the state (extensive totals Q and points X),
the scheme parameters, the time and the step count, written to one .npz
file (plain arrays, no pickled objects) and read back onto the device.

The mesh is not stored: it is the Voronoi tessellation of the points, which
the host input stage rebuilds from them exactly (exact predicates), so a
run resumed from step k on the rebuilt mesh continues bit for bit as the
uninterrupted run that tessellated the same points on the host.
"""
from __future__ import annotations

import json

import numpy as np

from . import rich as R

_FIELDS = ("gamma", "cfl", "theta", "delta_v", "delta_p", "chi", "eta", "riemann", "motion",
           "limiter", "gx", "gy", "integrator")
FORMAT = "rich-checkpoint-1"


def save(path, state: "R.DeviceState", params: "R.Params", t: float, step: int, box, bc):
    """Write the run to `path` (.npz).  Synchronises the device (copies the
    state to the host)."""
    Q, X = state.numpy()
    meta = {"format": FORMAT, "t": float(t), "step": int(step), "box": [float(v) for v in box],
            "bc": int(bc), "params": {k: getattr(params, k) for k in _FIELDS}}
    with open(path, "wb") as f:
        np.savez(f, Q=Q, X=X, meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load(path, device="cuda"):
    """(state on the device, Params, t, step, box, bc) of a checkpoint."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        if meta.get("format") != FORMAT:
            raise ValueError(f"{path}: not a {FORMAT} file")
        Q = np.array(z["Q"], dtype=np.float64)
        X = np.array(z["X"], dtype=np.float64)
    if Q.ndim != 2 or Q.shape[0] != 4 or X.shape != (2, Q.shape[1]):
        raise ValueError(f"{path}: state arrays of shapes {Q.shape}, {X.shape}")
    params = R.Params(**meta["params"])
    state = R.DeviceState.from_host(Q, X, device=device)
    return state, params, meta["t"], meta["step"], tuple(meta["box"]), meta["bc"]


def resume(path, device_tess=False, n_threads=0, device="cuda"):
    """A step driver (rich.RichCtx) positioned at the checkpoint: the mesh of
    the stored points is built by the host stage and set as the current mesh.
    Returns (ctx, state, params, t, step)."""
    from . import tess as T
    state, params, t, step, box, bc = load(path, device=device)
    X = state.X.cpu().numpy()
    ctx = R.RichCtx(n_threads=n_threads, device_tess=device_tess)
    ctx.set_mesh(T.rich_tess_build(X[0], X[1], box, bc, n_threads=n_threads))
    return ctx, state, params, t, step
