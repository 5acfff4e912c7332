"""Shared helpers of the GPU parity tests: seeded cases, running one stage on
both sides, and the two error metrics.

Per conserved quantity k, per stage:
    err_k = max_i |Q_gpu[k,i] - Q_oracle[k,i]| / scale_k
with scale = max|M| for mass, max_i M_i (c_i + |v_i|) for both momenta,
max|E| for energy and the box size for the points.  The bar is 1e-12.

Per cell (cell_errors), so that a cell far below the domain's largest
values (the ambient gas of a point explosion holds 1e-11 of the blast cell's
energy) is held to its own magnitude:
    rel_ik = |Q_gpu[k,i] - Q_oracle[k,i]| / T_ik
    T_ik   = |Q_base[k,i]| + |Q_oracle[k,i]| + h sum_e L_e (|F_ek| + S_ek)
           (+ h |source_ik| with an external acceleration)
where the sum runs over the cell's edges, F_e is the oracle's flux of the
edge and S_e the magnitude of the terms a flux of the edge's two cells is
built from (with U = |v| + |w| + c, rho, p and e = rho U^2 / 2 + p/(gamma-1)
the larger of the two cells': rho U for mass, rho U^2 + p for momentum,
(e + p) U for energy).  T_ik is what a rounding error of the cell's update
is proportional to.  The bar is again 1e-12.
"""
import math

import numpy as np

import oracle as O
from paper_1410_3219_amd import inputs as I
from paper_1410_3219_amd import tess as T

TOL = 1e-12


def host_mesh(px, py, box, bc):
    return T.rich_tess_build(px, py, box, bc)


def case(name, k=24, riemann=0, limiter=0, motion=1, pass2=False, seed=1, g=(0.0, 0.0),
         integrator=0):
    """(mesh, Qsrc, Qbase, Xbase, h, oracle Params)."""
    if name == "sod":
        P = I.sod(k=k, seed=seed)
        m = host_mesh(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
    elif name == "sod_angle":
        P = I.sod(k=k, seed=seed, angle=0.7, gamma=1.4)
        m = host_mesh(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
    elif name == "wave":
        P = I.advected_wave(k=k, seed=seed)
        m = host_mesh(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
    elif name == "acoustic":
        P = I.acoustic_wave(k=k, seed=seed, amp=1e-3)
        m = host_mesh(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
    elif name == "sedov":
        P = I.sedov(k=k, seed=seed, lloyd_iters=2)
        m = host_mesh(P.px, P.py, P.box, P.bc)
        Q = I.sedov_state(P, m.area)
    elif name == "kh":
        P = I.kelvin_helmholtz(k=k, seed=seed)
        m = host_mesh(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
    elif name == "gresho":
        P = I.gresho(k=k, seed=seed)
        m = host_mesh(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
    else:
        raise ValueError(name)
    p = O.Params(gamma=P.gamma, riemann=riemann, limiter=limiter, motion=motion,
                 gx=g[0], gy=g[1], integrator=integrator)
    X = np.stack([m.px, m.py])
    dt, st = O.cfl_dt(m, Q, p)
    assert st == 0
    if integrator == 1:   # extrapolated fluxes: one full-step stage
        return m, Q, Q, X, dt, p
    if not pass2:
        return m, Q, Q, X, 0.5 * dt, p
    # second pass of a time-centred step: primitives from the half-step state
    # on the half-step mesh, update applied to the start-of-step state
    s1 = O.stage(m, Q, Q, X, 0.5 * dt, p)
    assert s1.status == 0
    mh = host_mesh(s1.X[0], s1.X[1], m.box, m.bc) if motion else m
    return mh, s1.Q, Q, X, dt, p


def gpu_params(p):
    from paper_1410_3219_amd import rich as R
    return R.Params(gamma=p.gamma, cfl=p.cfl, theta=p.theta, delta_v=p.delta_v,
                    delta_p=p.delta_p, chi=p.chi, eta=p.eta, riemann=p.riemann,
                    motion=p.motion, limiter=p.limiter, gx=p.gx, gy=p.gy,
                    integrator=p.integrator)


def gpu_stage(m, Qs, Qb, Xb, h, p, repeat=1):
    import torch
    from paper_1410_3219_amd import rich as R
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    base = R.DeviceState.from_host(Qb, Xb)
    ws = R.workspace(m.n_cells)
    outs = []
    for _ in range(repeat):
        out = R.DeviceState.empty_like(base)
        out.Q.fill_(float("nan"))
        out.X.fill_(float("nan"))
        R.rich_stage(dm, src, base, out, h, gpu_params(p), ws)
        flags = R.rich_stage_flags(ws)
        torch.cuda.synchronize()
        Q, X = out.numpy()
        outs.append((Q, X, flags))
    return outs if repeat > 1 else outs[0]


def scales(m, Q, p, box):
    prim = O.primitives(m, Q, p)
    c = prim[4]
    v = np.hypot(prim[1], prim[2])
    return np.array([np.max(np.abs(Q[0])), np.max(Q[0] * (c + v)), np.max(Q[0] * (c + v)),
                     np.max(np.abs(Q[3]))]), max(box[2] - box[0], box[3] - box[1])


def errors(m, Qg, Xg, Qo, Xo, Qref, p):
    sc, L = scales(m, Qref, p, m.box)
    eq = np.max(np.abs(Qg - Qo), axis=1) / sc
    dx = np.abs(Xg - Xo)
    if m.bc == 1:
        dx = np.minimum(dx, L - dx)
    ex = np.max(dx) / L
    return eq, ex


def cell_scale(m, Qb, Qo, h, p, diag, Qs=None, accel=None):
    """T (4, n) of the per-cell metric.  Qo is the oracle's result; `diag`
    an oracle stage result with diagnostics (O.stage(..., diag=True):
    primitives, w, edge fluxes), which do not depend on the acceleration."""
    assert diag.prim is not None and diag.flux is not None, "needs O.stage(..., diag=True)"
    rho, vx, vy, pr, c = diag.prim
    w = diag.w
    U = np.hypot(vx, vy) + np.hypot(w[0], w[1]) + c
    e = 0.5 * rho * U * U + pr / (p.gamma - 1.0)
    ei = np.asarray(m.e_i, dtype=np.int64)
    ej32 = np.asarray(m.e_j).view(np.uint32)
    code = (ej32 >> 28).astype(np.int64)
    ej = (ej32 & 0x0FFFFFFF).astype(np.int64)
    inner = code < 9
    jj = np.where(inner, ej, ei)
    Ue = np.maximum(U[ei], U[jj])
    Re = np.maximum(rho[ei], rho[jj])
    Pe = np.maximum(pr[ei], pr[jj])
    Ee = np.maximum(e[ei], e[jj])
    S = [Re * Ue, Re * Ue * Ue + Pe, Re * Ue * Ue + Pe, (Ee + Pe) * Ue]
    L = np.asarray(m.e_len)
    n = Qb.shape[1]
    T = np.abs(Qb) + np.abs(Qo)
    for k in range(4):
        t = L * (np.abs(diag.flux[k]) + S[k])
        T[k] += h * (np.bincount(ei, t, minlength=n) +
                     np.bincount(ej[inner], t[inner], minlength=n))
    g = np.array([p.gx, p.gy], dtype=np.float64)[:, None] * np.ones((1, n))
    if accel is not None:
        g = g + accel
    if np.any(g != 0.0):
        Qs = Qb if Qs is None else Qs
        gm = np.hypot(g[0], g[1])
        T[1] += h * np.abs(Qs[0]) * gm
        T[2] += h * np.abs(Qs[0]) * gm
        T[3] += h * (np.abs(Qs[1]) + np.abs(Qs[2])) * gm
    return T


def cell_errors(m, Qg, Qb, Qo, h, p, diag, Qs=None, accel=None):
    """Largest per-cell relative difference of each conserved quantity
    (the per-cell metric above) and the cell where it occurs."""
    T = cell_scale(m, Qb, Qo, h, p, diag, Qs=Qs, accel=accel)
    r = np.abs(Qg - Qo) / T
    return r.max(axis=1), r.argmax(axis=1)


def check_stage(m, Qs, Qb, Xb, h, p, Qg, Xg, ref=None, accel=None, label=""):
    """Both bars for one stage: the per-quantity metric and the per-cell one.
    `ref` may be the oracle's stage result (with or without diagnostics).
    Returns (eq, ex, ec): per-quantity errors, point error, per-cell errors."""
    if ref is None:
        ref = (O.stage(m, Qs, Qb, Xb, h, p, diag=True) if accel is None else
               O.stage_accel(m, Qs, Qb, Xb, h, p, accel))
    assert ref.status == 0
    diag = ref if ref.flux is not None else O.stage(m, Qs, Qb, Xb, h, p, diag=True)
    eq, ex = errors(m, Qg, Xg, ref.Q, ref.X, Qb, p)
    ec, where = cell_errors(m, Qg, Qb, ref.Q, h, p, diag, Qs=Qs, accel=accel)
    print(f"\n{label} n={m.n_cells} err M,Px,Py,E={eq} x={ex:.2e} per-cell={ec} "
          f"at cells {where}", flush=True)
    assert (eq < TOL).all(), (label, eq)
    assert ex < TOL, (label, ex)
    assert (ec < TOL).all(), (label, ec, where)
    return eq, ex, ec
