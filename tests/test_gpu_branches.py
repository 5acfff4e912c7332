"""Branch records of a stage (rich_stage_debug) against the oracle's decisions.

Per cell: the shock flag of the switching limiter, the cell-rounding
correction and alpha < 1 for each field (section 2.2, section 6); per edge
the sign tests that pick the Riemann solver's branch (section 2.4).  Both
sides take each decision in FP64 from values that agree to rounding, so a
decision may differ only where the oracle's value lies within 1e-12
(relative) of its threshold: for alpha < 1, where min psi is within 1e-12
of 1, or where all of a cell's projected changes G.(f - s) are at rounding
level (a uniform region, whose gradient is noise: there alpha G is noise
whatever alpha is).  Such cells and edges are counted and reported, and
every other record must agree exactly.  The debug stage's outputs equal
rich_stage's bit for bit."""
import numpy as np
import pytest

import oracle as O
import parity_util as U

pytestmark = pytest.mark.gpu

MARGIN = 1e-12
MASK = (1 << 28) - 1


def _neighbours(m):
    """Per CSR entry: (owning cell, neighbour cell; a wall's mirror is the
    cell itself)."""
    idx = m.idx.astype(np.int64)
    e, side = idx >> 1, idx & 1
    ej = m.e_j.view(np.uint32).astype(np.int64)
    code = ej[e] >> 28
    j = np.where(side == 0, ej[e] & MASK, m.e_i.astype(np.int64)[e])
    cell = np.repeat(np.arange(m.n_cells), np.diff(m.off.astype(np.int64)))
    j = np.where((side == 0) & (code >= 9), cell, j)
    return cell, j


def _entries(m, prim):
    """Per CSR entry: (cell, edge midpoint minus the cell's centroid in the
    cell's own frame, the neighbour's rho, vx, vy, p; a wall's mirror has the
    cell's values with the normal velocity reversed)."""
    idx = m.idx.astype(np.int64)
    e, side = idx >> 1, idx & 1
    ej = m.e_j.view(np.uint32).astype(np.int64)
    code = ej[e] >> 28
    k = np.where(code <= 4, code - 1, code)
    Lx, Ly = m.box[2] - m.box[0], m.box[3] - m.box[1]
    periodic = (code >= 1) & (code <= 8) & (side == 1)
    shx = np.where(periodic, (k // 3 - 1) * Lx, 0.0)
    shy = np.where(periodic, (k % 3 - 1) * Ly, 0.0)
    cell = np.repeat(np.arange(m.n_cells), np.diff(m.off.astype(np.int64)))
    wall = (side == 0) & (code >= 9)
    j = np.where(side == 0, ej[e] & MASK, m.e_i.astype(np.int64)[e])
    j = np.where(wall, cell, j)
    phj = prim[:4, j].copy()
    phj[1] = np.where(wall & (code <= 10), -phj[1], phj[1])
    phj[2] = np.where(wall & (code >= 11), -phj[2], phj[2])
    return cell, m.e_fx[e] - shx - m.sx[cell], m.e_fy[e] - shy - m.sy[cell], phj


def _alpha_margin(m, prim, grad, flag, p):
    """How far each field's limiter decision alpha < 1 is from its threshold:
    |min_j psi_ij - 1| with the unclamped psi of the limiter in use, and 0
    (undecided) where every projected change G.(f - s) of the cell is at
    rounding level against the field's scale (a uniform region, whose
    gradient is rounding noise, as is alpha G whatever alpha is)."""
    n = m.n_cells
    out = np.full((4, n), np.inf)
    below = np.zeros((4, n), bool)
    if p.limiter in (3, 4):
        return out, below
    ce, ox, oy, phj = _entries(m, prim)
    local = np.zeros(n, bool) if p.limiter == 1 else (
        np.ones(n, bool) if p.limiter == 2 else (flag & 1).astype(bool))
    speed = np.hypot(prim[1], prim[2]) + prim[4]
    scale = [np.abs(prim[0]).max(), speed.max(), speed.max(), np.abs(prim[3]).max()]
    for q in range(4):
        phi = prim[q]
        pmax, pmin = phi.copy(), phi.copy()
        np.maximum.at(pmax, ce, phj[q])
        np.minimum.at(pmin, ce, phj[q])
        dphi = grad[2 * q][ce] * ox + grad[2 * q + 1][ce] * oy
        with np.errstate(divide="ignore", invalid="ignore"):
            glob = np.where(dphi > 0, (pmax[ce] - phi[ce]) / dphi,
                            np.where(dphi < 0, (pmin[ce] - phi[ce]) / dphi, 1.0))
            loc = np.where(dphi != 0, np.maximum(p.theta * (phj[q] - phi[ce]) / dphi, 0.0), 1.0)
        psi = np.where(local[ce], loc, glob)
        pmin_psi = np.full(n, np.inf)
        np.minimum.at(pmin_psi, ce, psi)
        dmax = np.zeros(n)
        np.maximum.at(dmax, ce, np.abs(dphi))
        out[q] = np.where(dmax < MARGIN * scale[q], 0.0, np.abs(pmin_psi - 1.0))
        below[q] = pmin_psi < 1.0
    return out, below


def _oracle_records(m, Qs, p):
    prim = O.primitives(m, Qs, p)
    w = O.point_velocity(m, prim, p)
    grad = O.gradients(m, prim)
    alpha, flag = O.limiter(m, prim, grad, p)
    lgrad = grad * np.repeat(alpha, 2, axis=0)
    waves, st = O.edge_waves(m, prim, lgrad, w, p)
    assert st == 0
    n = m.n_cells
    # cell bits
    d = np.hypot(m.sx - m.px, m.sy - m.py)
    R = np.sqrt(m.area / np.pi)
    rounded = (d > p.eta * R) if p.motion else np.zeros(n, bool)
    bits = (flag & 1).astype(np.int64) | (rounded.astype(np.int64) << 1)
    for q in range(4):
        bits |= (alpha[q] < 1.0).astype(np.int64) << (2 + q)
    # margins of each cell decision
    m_round = np.abs(d - p.eta * R) / (p.eta * R) if p.motion else np.full(n, np.inf)
    thr = p.delta_v * prim[4] / R
    m_comp = np.abs(-(grad[2] + grad[5]) - thr) / thr
    cell, j = _neighbours(m)
    pi, pj = prim[3][cell], prim[3][j]
    ratio = np.minimum(pi, pj) / np.maximum(pi, pj)
    m_pj = np.full(n, np.inf)
    np.minimum.at(m_pj, cell, np.abs(ratio - p.delta_p) / p.delta_p)
    m_shock = np.minimum(m_comp, m_pj)
    m_alpha, below = _alpha_margin(m, prim, grad, flag, p)
    # where it calls the decision settled, the margin's psi gives the
    # oracle's own alpha < 1
    if p.limiter not in (3, 4):
        settled = m_alpha > MARGIN
        assert ((alpha < 1.0) == below)[settled].all()
    # edge bits and margins
    sl, ss, sr, scale = waves
    if p.riemann == 0:
        ebits = ((0.0 <= sl).astype(np.int64) | ((0.0 <= ss).astype(np.int64) << 1)
                 | ((0.0 < sr).astype(np.int64) << 2))
        m_edge = np.stack([np.abs(sl), np.abs(ss), np.abs(sr)]) / scale
    else:
        ebits = (0.0 <= ss).astype(np.int64) << 1
        m_edge = (np.abs(ss) / scale)[None, :]
    return bits, (m_shock, m_round, m_alpha), ebits, m_edge


def _gpu_records(m, Qs, Qb, Xb, h, p):
    import torch
    from paper_1410_3219_amd import rich as R
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    base = R.DeviceState.from_host(Qb, Xb)
    ws = R.workspace(m.n_cells)
    out = R.DeviceState.empty_like(base)
    cb, eb = R.rich_stage_debug(dm, src, base, out, h, U.gpu_params(p), ws)
    flags = R.rich_stage_flags(ws)
    torch.cuda.synchronize()
    return cb.cpu().numpy().astype(np.int64), eb.cpu().numpy().astype(np.int64), out.numpy(), flags


CASES = [("sod", 24, 0, 0, 1, False), ("sod", 23, 0, 0, 1, True), ("sedov", 30, 0, 0, 1, True),
         ("kh", 26, 0, 0, 1, False), ("wave", 28, 0, 0, 1, True), ("gresho", 25, 0, 2, 1, False),
         ("sod_angle", 21, 1, 0, 1, True), ("sedov", 20, 1, 1, 1, False),
         ("kh", 18, 0, 3, 0, False), ("sod", 16, 0, 4, 1, False), ("wave", 26, 0, 0, 0, False)]


@pytest.mark.parametrize("name,k,riemann,limiter,motion,pass2", CASES)
def test_branch_records_match_oracle(name, k, riemann, limiter, motion, pass2):
    m, Qs, Qb, Xb, h, p = U.case(name, k=k, riemann=riemann, limiter=limiter, motion=motion,
                                 pass2=pass2)
    cb, eb, (Qd, Xd), flags = _gpu_records(m, Qs, Qb, Xb, h, p)
    assert flags == 0
    Qg, Xg, fg = U.gpu_stage(m, Qs, Qb, Xb, h, p)
    assert np.array_equal(Qd, Qg) and np.array_equal(Xd, Xg)
    bits, (m_shock, m_round, m_alpha), ebits, m_edge = _oracle_records(m, Qs, p)
    diff = cb ^ bits
    # shock flag
    bad = (diff & 1) != 0
    assert (m_shock[bad] < MARGIN).all(), np.flatnonzero(bad & (m_shock >= MARGIN))[:10]
    near_switch = bad.copy()   # the limiter itself changes in such cells
    # rounding
    bad = (diff & 2) != 0
    assert (m_round[bad] < MARGIN).all()
    # alpha < 1 per field
    for q in range(4):
        bad = (diff >> (2 + q) & 1) != 0
        ok = (m_alpha[q] < MARGIN) | near_switch
        assert ok[bad].all(), (q, np.flatnonzero(bad & ~ok)[:10])
    # Riemann branch; an edge of a cell whose limiter switched sees other face states
    ediff = eb ^ ebits
    assert not (eb & 8).any()
    ej = m.e_j.view(np.uint32).astype(np.int64)
    jn = np.where(ej >> 28 >= 9, m.e_i, ej & MASK)
    switched = near_switch[m.e_i] | near_switch[jn]
    if riemann == 0:
        for b in range(3):
            bad = (ediff >> b & 1) != 0
            ok = (m_edge[b] < MARGIN) | switched
            assert ok[bad].all(), (b, np.flatnonzero(bad & ~ok)[:10])
    else:
        bad = (ediff >> 1 & 1) != 0
        ok = (m_edge[0] < MARGIN) | switched
        assert ok[bad].all()
        assert not (eb & 5).any()
    n_cell_diff = int((diff != 0).sum())
    n_edge_diff = int((ediff != 0).sum())
    print(f"\n{name} k={k} riemann={riemann} limiter={limiter} pass2={pass2}: "
          f"shock {int((bits & 1).sum())}/{m.n_cells}, rounded {int((bits >> 1 & 1).sum())}, "
          f"alpha<1 {[int((bits >> (2 + q) & 1).sum()) for q in range(4)]}, "
          f"records differing within the margin: {n_cell_diff} cells, {n_edge_diff} edges")


def test_branch_records_are_not_vacuous():
    """Across a shock tube, a blast wave and shear flow every cell bit is
    seen set and clear, and a supersonic flow over a static mesh makes HLLC
    take all four branches."""
    seen_set = np.zeros(6, bool)
    seen_clear = np.zeros(6, bool)
    for name, k, pass2 in (("sod", 24, True), ("sedov", 30, True), ("kh", 26, False)):
        m, Qs, Qb, Xb, h, p = U.case(name, k=k, pass2=pass2)
        cb, eb, _, _ = _gpu_records(m, Qs, Qb, Xb, h, p)
        for b in range(6):
            seen_set[b] |= bool((cb >> b & 1).any())
            seen_clear[b] |= bool((~cb >> b & 1).any())
    assert seen_set.all() and seen_clear.all(), (seen_set, seen_clear)
    m, Qs, Qb, Xb, h, p = U.case("wave", k=26, motion=0)
    _, eb, _, _ = _gpu_records(m, Qs, Qb, Xb, h, p)
    branches = set(np.unique(eb).tolist())
    assert branches == {0, 4, 6, 7}, branches   # F_R, F*_R, F*_L, F_L


def test_debug_stage_invalid_arguments():
    import ctypes as C
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("sod", k=8)
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    base = R.DeviceState.from_host(Qb, Xb)
    out = R.DeviceState.empty_like(base)
    ws = R.workspace(m.n_cells)
    st = R.lib().rich_stage_debug(C.byref(dm.c()), C.byref(src.c()), C.byref(base.c()),
                                  C.byref(out.c()), float(h), C.byref(U.gpu_params(p).c()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), None, None, None)
    assert st == R.RICH_E_INVAL
