"""Device re-tessellation (rich_retess) through the C-ABI.

The reference for the cells is the oracle's Voronoi tessellation by
definition (or_voronoi, clipping against every point) on small meshes, and
the exact-predicate Delaunay construction of the input stage at full size.
Topology (each cell's kept neighbours with their image / wall codes) must be
identical; areas, centroids, edge lengths and midpoints agree to 1e-12 of the
cell size.  Stages and time-centred chains on device-built meshes follow the
oracle on oracle-built meshes to the stage bar."""
import math

import numpy as np
import pytest

import oracle as O
import parity_util as U
from paper_1410_3219_amd import inputs as I
from paper_1410_3219_amd import tess as T

pytestmark = pytest.mark.gpu

MASK = 0x0FFFFFFF


def csr_keys(h):
    """Per CSR entry: (cell, neighbour, code seen from the cell) as one int64,
    sorted, and the edge length in the same order."""
    n = h.n_cells
    off = np.asarray(h.off, dtype=np.int64)
    cell = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    ent = np.asarray(h.idx[: off[-1]], dtype=np.int64)
    e, side = ent >> 1, ent & 1
    u = np.asarray(h.e_j, dtype=np.int64)[e] & 0xFFFFFFFF
    jc, code = u & MASK, u >> 28
    nb = np.where(side == 0, jc, np.asarray(h.e_i, dtype=np.int64)[e])
    cd = np.where(side == 0, code, np.where(code == 0, 0, 9 - code))
    key = (cell << 36) | (nb << 4) | cd
    o = np.argsort(key, kind="stable")
    return key[o], np.asarray(h.e_len)[e][o]


def edge_keys(h):
    """Per edge (owner side): key, length, midpoint, sorted by key."""
    ne = h.n_edges
    ei = np.asarray(h.e_i[:ne], dtype=np.int64)
    u = np.asarray(h.e_j[:ne], dtype=np.int64) & 0xFFFFFFFF
    key = (ei << 36) | ((u & MASK) << 4) | (u >> 28)
    o = np.argsort(key, kind="stable")
    return key[o], np.asarray(h.e_len[:ne])[o], np.asarray(h.e_fx[:ne])[o], \
        np.asarray(h.e_fy[:ne])[o]


def check_structure(h):
    """CSR and edge arrays are well formed: offsets monotone, edges sorted by
    owner with eoff, every CSR entry names an edge of its cell."""
    n = h.n_cells
    off, eoff = np.asarray(h.off), np.asarray(h.eoff)
    assert off[0] == 0 and eoff[0] == 0
    assert (np.diff(off) >= 0).all() and (np.diff(eoff) >= 0).all()
    assert off[-1] == h.n_csr and eoff[-1] == h.n_edges
    ei = np.asarray(h.e_i[: h.n_edges])
    assert (ei == np.repeat(np.arange(n), np.diff(eoff))).all()
    cell = np.repeat(np.arange(n), np.diff(off))
    ent = np.asarray(h.idx[: h.n_csr])
    e, side = ent >> 1, ent & 1
    assert (e >= 0).all() and (e < h.n_edges).all()
    u = np.asarray(h.e_j, dtype=np.int64)[e] & 0xFFFFFFFF
    other = np.where(side == 0, ei[e], u & MASK)
    assert (other == cell).all()
    assert (2 * h.n_edges - np.count_nonzero(
        (np.asarray(h.e_j[: h.n_edges], dtype=np.int64) & 0xFFFFFFFF) >> 28 >= 9)
        == h.n_csr)


def compare_meshes(dev, ref, h_cell, tol=1e-12):
    """Same topology, geometry within tol * cell size."""
    assert dev.n_edges == ref.n_edges and dev.n_csr == ref.n_csr
    kd, ld = csr_keys(dev)
    kr, lr = csr_keys(ref)
    assert np.array_equal(kd, kr)
    assert np.abs(ld - lr).max() <= tol * h_cell
    ed, edl, edx, edy = edge_keys(dev)
    er, erl, erx, ery = edge_keys(ref)
    assert np.array_equal(ed, er)
    assert np.abs(edl - erl).max() <= tol * h_cell
    assert np.abs(edx - erx).max() <= tol * h_cell and np.abs(edy - ery).max() <= tol * h_cell
    assert np.abs(dev.area - ref.area).max() <= tol * h_cell * h_cell
    assert np.abs(dev.sx - ref.sx).max() <= tol * h_cell
    assert np.abs(dev.sy - ref.sy).max() <= tol * h_cell
    assert np.array_equal(dev.px, ref.px) and np.array_equal(dev.py, ref.py)


def _problem(name, k, seed=1):
    if name == "sod":
        return I.sod(k=k, seed=seed)
    if name == "wave":
        return I.advected_wave(k=k, seed=seed)
    if name == "sedov":
        return I.sedov(k=k, seed=seed, lloyd_iters=2)
    if name == "kh":
        return I.kelvin_helmholtz(k=k, seed=seed)
    if name == "gresho":
        return I.gresho(k=k, seed=seed)
    raise ValueError(name)


def _initial(name, k, seed=1):
    P = _problem(name, k, seed)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = I.sedov_state(P, m.area) if name == "sedov" else P.state(m.area)
    return P, m, Q, np.stack([m.px, m.py])


def _half_step_points(R, dm, Q, X, p):
    """Points after a real stage-1 move (device)."""
    s = R.DeviceState.from_host(Q, X)
    half = R.DeviceState.empty_like(s)
    ws = R.workspace(dm.n_cells)
    R.rich_stage_courant(dm, s, s, half, 0.5, p, ws)
    assert R.rich_stage_flags(ws) == 0
    return s, half


@pytest.mark.parametrize("name,k", [("sod", 24), ("wave", 27), ("sedov", 26), ("kh", 22),
                                    ("gresho", 20)])
def test_retess_matches_oracle_voronoi(name, k):
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _initial(name, k)
    dm = R.DeviceMesh.from_host(m)
    p = R.Params(gamma=P.gamma, motion=1)
    s, half = _half_step_points(R, dm, Q, X, p)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    R.rich_retess(dm, half.X, bufs, tws)
    st, info = R.rich_retess_result(tws)
    assert st == 0 and info["flags"] == 0 and info["sticky"] == 0, info
    dev = R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"])
    check_structure(dev)
    Xh = half.X.cpu().numpy()
    ref = O.voronoi_mesh(O.voronoi(Xh[0], Xh[1], m.box, m.bc))
    h_cell = math.sqrt((m.box[2] - m.box[0]) * (m.box[3] - m.box[1]) / m.n_cells)
    compare_meshes(dev, ref, h_cell)
    assert abs(info["area_sum"] - (m.box[2] - m.box[0]) * (m.box[3] - m.box[1])) < 1e-12


@pytest.mark.parametrize("petals,box", [(12, "walls"), (14, "walls"), (16, "walls"),
                                         (13, "periodic")])
def test_retess_wide_cells_match_oracle_voronoi(petals, box):
    """A cell with more candidates than the first clip launch holds (a point
    inside a ring of 12 to 16): it is left to the wide launch, and the mesh
    is certified and equals the oracle's Voronoi cells; the rest of the mesh
    comes from the first launch."""
    from paper_1410_3219_amd import rich as R
    P = I.sod(k=20, seed=4) if box == "walls" else I.advected_wave(k=20, seed=4)
    keep = np.hypot(P.px - 0.5, P.py - 0.5) > 0.1
    a = 2 * np.pi * np.arange(petals) / petals
    px = np.concatenate([P.px[keep], [0.5], 0.5 + 0.06 * np.cos(a)])
    py = np.concatenate([P.py[keep], [0.5], 0.5 + 0.06 * np.sin(a)])
    m = T.rich_tess_build(px, py, P.box, P.bc)
    assert np.diff(m.off).max() == petals
    dm = R.DeviceMesh.from_host(m)
    X = torch_points(R, m)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    R.rich_retess(dm, X, bufs, tws)
    st, info = R.rich_retess_result(tws)
    assert st == 0 and info["flags"] == 0, info
    dev = R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"])
    check_structure(dev)
    assert np.diff(dev.off).max() == petals
    ref = O.voronoi_mesh(O.voronoi(m.px, m.py, m.box, m.bc))
    h_cell = math.sqrt((m.box[2] - m.box[0]) * (m.box[3] - m.box[1]) / m.n_cells)
    compare_meshes(dev, ref, h_cell)


def torch_points(R, m):
    import torch
    return torch.from_numpy(np.stack([m.px, m.py])).cuda()


@pytest.mark.parametrize("name", ["sod", "wave"])
def test_retess_after_edge_flips_matches_oracle_voronoi(name):
    """Points jostled by up to a fifth of the spacing from the previous
    mesh's points: many previous neighbours no longer share an edge (their
    candidates bound nothing, and the positions they took in a cell's
    counter-clockwise order are closed up), new neighbours enter from the
    second ring; the result is still the oracle's Voronoi mesh."""
    from paper_1410_3219_amd import rich as R
    import torch
    P, m, Q, X = _initial(name, 24)
    h = math.sqrt((m.box[2] - m.box[0]) * (m.box[3] - m.box[1]) / m.n_cells)
    d = np.random.default_rng(5).uniform(-0.2 * h, 0.2 * h, X.shape)
    X1 = X + d
    if m.bc == 1:
        X1 = np.stack([np.mod(X1[0] - m.box[0], m.box[2] - m.box[0]) + m.box[0],
                       np.mod(X1[1] - m.box[1], m.box[3] - m.box[1]) + m.box[1]])
    else:
        X1 = np.stack([np.clip(X1[0], m.box[0] + 1e-3 * h, m.box[2] - 1e-3 * h),
                       np.clip(X1[1], m.box[1] + 1e-3 * h, m.box[3] - 1e-3 * h)])
    dm = R.DeviceMesh.from_host(m)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    R.rich_retess(dm, torch.from_numpy(np.ascontiguousarray(X1)).cuda(), bufs, tws)
    st, info = R.rich_retess_result(tws)
    assert st == 0 and info["flags"] == 0, info
    dev = R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"])
    check_structure(dev)
    ref = O.voronoi_mesh(O.voronoi(X1[0], X1[1], m.box, m.bc))
    compare_meshes(dev, ref, h)
    lost = np.setdiff1d(csr_keys(m)[0], csr_keys(ref)[0])
    gained = np.setdiff1d(csr_keys(ref)[0], csr_keys(m)[0])
    print(f"\n{name}: {lost.size} CSR entries lost, {gained.size} gained, "
          f"{info['n_clipped']} of {m.n_cells} cells clipped")
    assert lost.size > 20 and gained.size > 20
    # both paths ran: the cells that kept their ring were proved by the
    # vertex check, the others clipped
    assert 0 < info["n_clipped"] < m.n_cells


@pytest.mark.parametrize("name", ["wave", "sod"])
def test_retess_vertex_check_proves_unchanged_rings(name):
    """Cells that keep their previous neighbours are proved by the vertex
    check alone: after a rigid translation of the periodic wave's points no
    cell is clipped; on the walled shock tube's own points only the cells
    with a wall edge (which the check leaves to the clip) and at most 1% more
    are.  Either way the mesh is the oracle's Voronoi mesh."""
    from paper_1410_3219_amd import rich as R
    import torch
    P, m, Q, X = _initial(name, 32)
    L = (m.box[2] - m.box[0], m.box[3] - m.box[1])
    h = math.sqrt(L[0] * L[1] / m.n_cells)
    if m.bc == 1:
        X1 = np.stack([np.mod(X[0] + 0.37 * h - m.box[0], L[0]) + m.box[0],
                       np.mod(X[1] + 0.21 * h - m.box[1], L[1]) + m.box[1]])
    else:
        X1 = X.copy()
    dm = R.DeviceMesh.from_host(m)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    R.rich_retess(dm, torch.from_numpy(np.ascontiguousarray(X1)).cuda(), bufs, tws)
    st, info = R.rich_retess_result(tws)
    assert st == 0 and info["flags"] == 0, info
    dev = R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"])
    check_structure(dev)
    ref = O.voronoi_mesh(O.voronoi(X1[0], X1[1], m.box, m.bc))
    compare_meshes(dev, ref, h)
    if m.bc == 1:
        assert info["n_clipped"] == 0, info
    else:
        walled = np.unique(np.asarray(m.e_i)[m.nb_code() >= 9]).size
        assert walled > 0
        assert walled <= info["n_clipped"] <= walled + m.n_cells // 100, (walled, info)


@pytest.mark.parametrize("k", [4, 5, 8])
def test_retess_small_periodic_boxes_match_oracle_voronoi(k):
    """The smallest periodic boxes the device rebuild takes (16 cells and
    up): every cell is near the box's edges, so every wave seeks periodic
    images, and a cell's candidates can hold two images of one cell.  Both
    the points of the previous mesh and points moved by up to a tenth of the
    spacing give the oracle's Voronoi mesh."""
    from paper_1410_3219_amd import rich as R
    import torch
    P, m, Q, X = _initial("wave", k, seed=3)
    L = (m.box[2] - m.box[0], m.box[3] - m.box[1])
    h = math.sqrt(L[0] * L[1] / m.n_cells)
    d = np.random.default_rng(k).uniform(-0.1 * h, 0.1 * h, X.shape)
    for X1 in (X, X + d):
        X1 = np.stack([np.mod(X1[0] - m.box[0], L[0]) + m.box[0],
                       np.mod(X1[1] - m.box[1], L[1]) + m.box[1]])
        dm = R.DeviceMesh.from_host(m)
        bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
        tws = R.retess_workspace(m.n_cells)
        R.rich_retess(dm, torch.from_numpy(np.ascontiguousarray(X1)).cuda(), bufs, tws)
        st, info = R.rich_retess_result(tws)
        assert st == 0 and info["flags"] == 0, info
        dev = R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"])
        check_structure(dev)
        ref = O.voronoi_mesh(O.voronoi(X1[0], X1[1], m.box, m.bc))
        compare_meshes(dev, ref, h)


def test_retess_repeat_is_bitwise_deterministic():
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _initial("sedov", 30)
    dm = R.DeviceMesh.from_host(m)
    p = R.Params(gamma=P.gamma)
    s, half = _half_step_points(R, dm, Q, X, p)
    outs = []
    for _ in range(2):
        bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
        tws = R.retess_workspace(m.n_cells)
        R.rich_retess(dm, half.X, bufs, tws)
        assert R.rich_retess_result(tws)[0] == 0
        outs.append({k: v.cpu() for k, v in bufs.t.items()})
    for k in outs[0]:
        if k in ("edges", "idx"):
            continue
        assert np.array_equal(outs[0][k].numpy(), outs[1][k].numpy()), k
    st, info = R.rich_retess_result(tws)
    ne, nc = info["n_edges"], info["n_csr"]
    assert np.array_equal(outs[0]["edges"][: 32 * ne].numpy(), outs[1]["edges"][: 32 * ne].numpy())
    assert np.array_equal(outs[0]["idx"][:nc].numpy(), outs[1]["idx"][:nc].numpy())


@pytest.mark.parametrize("name,k", [("wave", 100), ("sod", 90)])
def test_retess_sums_reproducible_over_many_blocks(name, k):
    """The result header's area sum and dropped-edge count come from per-block
    sums reduced in a fixed order (over several scan blocks of 1024 cells
    here): two calls give the same bits, the area sum equals the box area and
    the cells' own areas summed on the host to rounding, and the kept CSR
    entries are twice the edges less the wall edges."""
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _initial(name, k)
    assert m.n_cells > 4 * 1024
    dm = R.DeviceMesh.from_host(m)
    p = R.Params(gamma=P.gamma)
    s, half = _half_step_points(R, dm, Q, X, p)
    infos, areas = [], []
    for _ in range(2):
        bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
        tws = R.retess_workspace(m.n_cells)
        R.rich_retess(dm, half.X, bufs, tws)
        st, info = R.rich_retess_result(tws)
        assert st == 0, info
        infos.append(info)
        cells = bufs.t["cells"].cpu().numpy().view(np.float64).reshape(-1, 6)
        areas.append(cells[:, 2].copy())
    assert infos[0] == infos[1]
    assert np.array_equal(areas[0], areas[1])
    box = (m.box[2] - m.box[0]) * (m.box[3] - m.box[1])
    a_host = float(np.sum(areas[0]))
    assert abs(infos[0]["area_sum"] - a_host) <= 1e-13 * box, (infos[0]["area_sum"], a_host)
    assert abs(infos[0]["area_sum"] - box) <= 1e-10 * box
    edges = bufs.t["edges"][: R.EDGE_BYTES * infos[0]["n_edges"]].cpu().numpy()
    codes = edges.view(np.int32).reshape(-1, 8)[:, 7].view(np.uint32) >> 28
    n_wall = int(np.count_nonzero(codes >= 9))
    assert infos[0]["n_csr"] == 2 * infos[0]["n_edges"] - n_wall


@pytest.mark.parametrize("name", ["sod", "wave", "sedov"])
def test_stage_on_device_mesh_matches_oracle(name):
    """Stage 2 of a time-centred step on the device-built half-step mesh
    against the oracle's stage on its own Voronoi mesh of the same points."""
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _initial(name, 26)
    dm = R.DeviceMesh.from_host(m)
    op = O.Params(gamma=P.gamma)
    p = U.gpu_params(op)
    ws = R.workspace(m.n_cells)
    s = R.DeviceState.from_host(Q, X)
    half = R.DeviceState.empty_like(s)
    R.rich_stage_courant(dm, s, s, half, 0.5, p, ws)
    dt = R.rich_stage_dt(ws)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    R.rich_retess(dm, half.X, bufs, tws)
    assert R.rich_retess_result(tws)[0] == 0
    out = R.DeviceState.empty_like(s)
    R.rich_stage_dt_of(bufs.mesh(), half, s, out, 1.0, ws, p, ws)
    assert R.rich_stage_flags(ws) == 0
    Qh, Xh = half.numpy()
    mo = O.voronoi_mesh(O.voronoi(Xh[0], Xh[1], m.box, m.bc))
    ref = O.stage(mo, Qh, Q, X, dt, op)
    assert ref.status == 0
    Qg, Xg = out.numpy()
    eq, ex = U.errors(mo, Qg, Xg, ref.Q, ref.X, Q, op)
    print(f"\n{name} stage 2 on device mesh: err {eq} x {ex}")
    assert (eq < U.TOL).all() and ex < U.TOL, (eq, ex)


@pytest.mark.parametrize("name", ["sod", "wave", "kh"])
def test_device_chain_follows_oracle_chain(name):
    """Four time-centred steps with every mesh after the first built on the
    device (Courant step on the device too) against the oracle's chain whose
    meshes are its own Voronoi tessellations."""
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _initial(name, 22)
    op = O.Params(gamma=P.gamma)
    p = U.gpu_params(op)
    n = m.n_cells

    def tess(px, py, box, bc):
        return O.voronoi_mesh(O.voronoi(px, py, box, bc))

    Qo, Xo, mo = Q, X, tess(m.px, m.py, m.box, m.bc)
    dts = []
    mesh = R.DeviceMesh.from_host(m)
    ws = R.workspace(n)
    s = R.DeviceState.from_host(Q, X)
    half = R.DeviceState.empty_like(s)
    nxt = R.DeviceState.empty_like(s)
    bufs = [R.DeviceMeshBufs(n, m.box, m.bc) for _ in range(3)]
    tws = R.retess_workspace(n)
    b = 0
    for step in range(4):
        R.rich_stage_courant(mesh, s, s, half, 0.5, p, ws)
        mh = bufs[b % 3]
        b += 1
        R.rich_retess(mesh, half.X, mh, tws)
        R.rich_stage_dt_of(mh.mesh(), half, s, nxt, 1.0, ws, p, ws)
        mn = bufs[b % 3]
        b += 1
        R.rich_retess(mh.mesh(), nxt.X, mn, tws)
        dts.append(R.rich_stage_dt(ws))
        mesh = mn.mesh()
        s, nxt = nxt, s
    st, info = R.rich_retess_result(tws)
    assert st == 0 and info["sticky"] == 0, info
    for dt in dts:
        Qo, Xo, mo, _, sto = O.step(mo, Qo, Xo, dt, op, tess)
        assert sto == 0
    Qg, Xg = s.numpy()
    eq, ex = U.errors(mo, Qg, Xg, Qo, Xo, Qo, op)
    print(f"\n{name} 4-step device chain err {eq} x {ex}")
    assert (eq < 1e-11).all() and ex < 1e-12


def test_retess_full_size_matches_host_stage():
    """The benchmark mesh (2048^2 = 4 194 304 cells, periodic) after a real
    half step: every cell, edge and CSR entry against the input stage's exact
    construction on the same points."""
    from paper_1410_3219_amd import rich as R
    P = I.advected_wave(k=2048, seed=1)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    dm = R.DeviceMesh.from_host(m)
    p = R.Params(gamma=P.gamma)
    s, half = _half_step_points(R, dm, Q, X, p)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    R.rich_retess(dm, half.X, bufs, tws)
    st, info = R.rich_retess_result(tws)
    assert st == 0, info
    dev = R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"])
    del bufs
    Xh = half.X.cpu().numpy()
    ref = T.rich_tess_build(Xh[0], Xh[1], P.box, P.bc)
    check_structure(dev)
    compare_meshes(dev, ref, 1.0 / 2048)


def test_retess_failure_is_reported_and_safe():
    """Candidates from a mesh of other points (every point moved by three
    cell sizes in a random direction): the certification fails, the output
    mesh has no edges, and a stage on it reads none."""
    from paper_1410_3219_amd import rich as R
    import torch
    P, m, Q, X = _initial("sod", 24)
    r = np.random.default_rng(3)
    h = 1.0 / 24
    ang = r.uniform(0, 2 * np.pi, m.n_cells)
    Xm = X + 3 * h * np.stack([np.cos(ang), np.sin(ang)])
    Xm = np.clip(Xm, 1e-3, 1 - 1e-3)
    dm = R.DeviceMesh.from_host(m)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    Xd = torch.from_numpy(Xm).cuda()
    R.rich_retess(dm, Xd, bufs, tws)
    st, info = R.rich_retess_result(tws)
    assert st == R.RICH_E_MESH and info["flags"] != 0, info
    assert info["sticky"] == info["flags"]
    assert (bufs.t["off"].cpu().numpy() == 0).all()
    assert (bufs.t["eoff"].cpu().numpy() == 0).all()
    # a stage on the failed mesh touches no edge and stays bounded
    s = R.DeviceState.from_host(Q, Xm)
    out = R.DeviceState.empty_like(s)
    ws = R.workspace(m.n_cells)
    R.rich_stage(bufs.mesh(), s, s, out, 1e-4, R.Params(gamma=P.gamma), ws)
    R.rich_stage_flags(ws)
    # the next good call clears the flags but not the sticky word
    R.rich_retess(dm, torch.from_numpy(X).cuda(), bufs, tws)
    st, info2 = R.rich_retess_result(tws)
    assert st == 0 and info2["flags"] == 0 and info2["sticky"] == info["flags"]


def test_retess_points_outside_reported():
    from paper_1410_3219_amd import rich as R
    import torch
    P, m, Q, X = _initial("wave", 20)
    Xb = X.copy()
    Xb[0, 5] = 1.5     # outside the periodic box
    dm = R.DeviceMesh.from_host(m)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    R.rich_retess(dm, torch.from_numpy(Xb).cuda(), bufs, tws)
    st, info = R.rich_retess_result(tws)
    assert st == R.RICH_E_MESH and info["flags"] & R.RETESS_POINT


def test_retess_invalid_arguments():
    from paper_1410_3219_amd import rich as R
    import torch
    P = I.advected_wave(k=3, seed=1)   # 9 cells in a periodic box: too few
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    dm = R.DeviceMesh.from_host(m)
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    tws = R.retess_workspace(m.n_cells)
    X = torch.from_numpy(np.stack([m.px, m.py])).cuda()
    with pytest.raises(R.RichError) as e:
        R.rich_retess(dm, X, bufs, tws)
    assert e.value.status == R.RICH_E_INVAL
    P, m, Q, Xh = _initial("sod", 10)
    dm = R.DeviceMesh.from_host(m)
    X = torch.from_numpy(Xh).cuda()
    small = R.retess_workspace(m.n_cells)[:1024]
    bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
    with pytest.raises(R.RichError) as e:
        R.rich_retess(dm, X, bufs, small)
    assert e.value.status == R.RICH_E_NOMEM
    other = R.DeviceMeshBufs(m.n_cells + 1, m.box, m.bc)
    with pytest.raises(R.RichError) as e:
        R.rich_retess(dm, X, other, R.retess_workspace(m.n_cells + 1))
    assert e.value.status == R.RICH_E_INVAL


@pytest.mark.parametrize("name", ["sod", "wave"])
def test_step_driver_with_device_tess_follows_oracle_chain(name):
    """rich_step with device re-tessellation: four steps, every mesh after
    the first built on the device, against the oracle chain on its own
    Voronoi meshes."""
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _initial(name, 22)
    op = O.Params(gamma=P.gamma)

    def tess(px, py, box, bc):
        return O.voronoi_mesh(O.voronoi(px, py, box, bc))

    dt, _ = O.cfl_dt(m, Q, op)
    ctx = R.RichCtx(device_tess=True)
    ctx.set_mesh(m)
    s = R.DeviceState.from_host(Q, X)
    Qo, Xo, mo = Q, X, tess(m.px, m.py, m.box, m.bc)
    for _ in range(4):
        ctx.step(s, dt, U.gpu_params(op))
        Qo, Xo, mo, _, sto = O.step(mo, Qo, Xo, dt, op, tess)
        assert sto == 0
    assert ctx.tess_counts() == (8, 0)
    Qg, Xg = s.numpy()
    eq, ex = U.errors(mo, Qg, Xg, Qo, Xo, Qo, op)
    print(f"\n{name} step driver, device meshes: err {eq} x {ex}")
    assert (eq < 1e-11).all() and ex < 1e-12
    ctx.close()


def test_step_driver_falls_back_to_host_stage():
    """A current mesh whose cells are other points (a permutation) gives the
    device re-tessellation wrong candidates: it is not certified, the host
    stage builds that mesh instead, and the step equals the host-only
    driver's bit for bit."""
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _initial("sod", 16)
    perm = np.random.default_rng(7).permutation(m.n_cells)
    mp = T.rich_tess_build(m.px[perm], m.py[perm], m.box, m.bc)
    Qu = I.conserved(1.0, 0.0, 0.0, 1.0, m.area, P.gamma)
    p = R.Params(gamma=P.gamma)
    out = []
    for dev in (True, False):
        ctx = R.RichCtx(device_tess=dev)
        ctx.set_mesh(mp)
        s = R.DeviceState.from_host(Qu, X)
        ctx.step(s, 1e-3, p)
        out.append((s.numpy(), ctx.tess_counts()))
        ctx.close()
    (Qd, Xd), counts = out[0]
    (Qh, Xh), counts_h = out[1]
    assert counts[1] >= 1 and counts_h == (0, 0), counts
    assert np.array_equal(Qd, Qh) and np.array_equal(Xd, Xh)


@pytest.mark.parametrize("bc", [0, 1])
def test_retess_exact_lattices(bc):
    """Degenerate inputs: an exact square lattice (four points on every
    Voronoi vertex's circle, so the diagonal edges have zero length and are
    dropped) and an exact hexagonal one, re-tessellated from a mesh of
    jittered points: the same cells as the oracle's Voronoi tessellation."""
    from paper_1410_3219_amd import rich as R
    import torch
    k = 24
    g = (np.arange(k) + 0.5) / k
    px, py = [a.ravel().copy() for a in np.meshgrid(g, g, indexing="ij")]
    box = (0.0, 0.0, 1.0, 1.0)
    r = np.random.default_rng(5)
    jx = px + 0.05 / k * r.uniform(-1, 1, px.size)
    jy = py + 0.05 / k * r.uniform(-1, 1, py.size)
    m = T.rich_tess_build(jx, jy, box, bc)
    dm = R.DeviceMesh.from_host(m)
    for (qx, qy, bx) in ((px, py, box), _hex(k, bc)):
        if bx != box:
            m2 = T.rich_tess_build(qx + 0.01 / k, qy, bx, bc)
            dprev = R.DeviceMesh.from_host(m2)
        else:
            dprev = dm
        bufs = R.DeviceMeshBufs(qx.size, bx, bc)
        tws = R.retess_workspace(qx.size)
        Xd = torch.from_numpy(np.stack([qx, qy])).cuda()
        R.rich_retess(dprev, Xd, bufs, tws)
        st, info = R.rich_retess_result(tws)
        assert st == 0, info
        dev = R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"])
        check_structure(dev)
        ref = O.voronoi_mesh(O.voronoi(qx, qy, bx, bc))
        compare_meshes(dev, ref, 1.0 / k)


def _hex(k, bc):
    """k x k hexagonal lattice (rows offset by half a spacing) in a box of
    height k * sqrt(3)/2 spacings; with walls, shifted off the walls."""
    a = 1.0 / k
    xs, ys = [], []
    for rr in range(k):
        for c in range(k):
            xs.append((c + 0.5 * (rr % 2) + 0.25) * a)
            ys.append((rr + 0.5) * a * math.sqrt(3.0) / 2.0)
    return np.array(xs), np.array(ys), (0.0, 0.0, 1.0, k * a * math.sqrt(3.0) / 2.0)


def test_retess_batch_equals_single_runs_bitwise():
    """rich_retess_batch over runs of different sizes and boundaries: every
    run's mesh and result equal its own rich_retess bit for bit; a run whose
    candidates are wrong fails alone."""
    from paper_1410_3219_amd import rich as R
    import torch
    cases = [("sod", 13), ("wave", 21), ("sedov", 17), ("kh", 9), ("gresho", 25)]
    prevs, Xs, ns = [], [], []
    for r, (name, k) in enumerate(cases):
        P, m, Q, X = _initial(name, k, seed=r + 2)
        dm = R.DeviceMesh.from_host(m)
        p = R.Params(gamma=P.gamma)
        _, half = _half_step_points(R, dm, Q, X, p)
        if r == 3:   # candidates from a mesh of permuted points: not certified
            perm = np.random.default_rng(1).permutation(m.n_cells)
            dm = R.DeviceMesh.from_host(T.rich_tess_build(m.px[perm], m.py[perm], m.box, m.bc))
        prevs.append(dm)
        Xs.append(half.X)
        ns.append(m.n_cells)
    single = []
    for dm, X, n in zip(prevs, Xs, ns):
        b = R.DeviceMeshBufs(n, dm.box, dm.bc)
        w = R.retess_workspace(n)
        R.rich_retess(dm, X, b, w)
        single.append((R.rich_retess_result(w), {k: v.cpu() for k, v in b.t.items()}))
    bufs = [R.DeviceMeshBufs(n, dm.box, dm.bc) for dm, n in zip(prevs, ns)]
    wss = [R.retess_workspace(n) for n in ns]
    bws = R.rich_retess_batch(prevs, Xs, bufs, wss)
    # the runs' flags without a wait: valid once the stream passes the copy
    hf = torch.full((len(prevs),), -1, dtype=torch.int32).pin_memory()
    R.rich_retess_batch_flags_async(len(prevs), bws, hf)
    ev = torch.cuda.Event()
    ev.record()
    ev.synchronize()
    res = R.rich_retess_batch_result(len(prevs), bws)
    assert [int(f) for f in hf] == [info["flags"] for _, info in res]
    assert [f != 0 for f in hf.tolist()] == [st == R.RICH_E_MESH for st, _ in res]

    def same(i1, i2):   # the area sum too: it is summed in a fixed order
        return dict(i1) == dict(i2)

    for r, ((st1, info1), t1) in enumerate(single):
        st2, info2 = res[r]
        assert st1 == st2 and same(info1, info2), (r, info1, info2)
        st3, info3 = R.rich_retess_result(wss[r])
        assert st3 == st2 and same(info3, info2)
        if r == 3:
            assert st2 == R.RICH_E_MESH
            continue
        assert st2 == 0
        ne, nc = info2["n_edges"], info2["n_csr"]
        t2 = {k: v.cpu() for k, v in bufs[r].t.items()}
        for key, lim in (("cells", None), ("off", None), ("eoff", None), ("edges", 32 * ne),
                         ("idx", nc)):
            a, b = t1[key].numpy(), t2[key].numpy()
            if lim is not None:
                a, b = a[:lim], b[:lim]
            assert np.array_equal(a, b), (r, key)


def test_step_driver_small_periodic_box_uses_host_stage():
    """A periodic box of 9 cells is below what the device rebuild takes: the
    driver builds those meshes with the host stage and the step equals the
    host-only driver's bit for bit."""
    from paper_1410_3219_amd import rich as R
    P = I.advected_wave(k=3, seed=2)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    p = R.Params(gamma=P.gamma)
    out = []
    for dev in (True, False):
        ctx = R.RichCtx(device_tess=dev)
        ctx.set_mesh(m)
        s = R.DeviceState.from_host(Q, X)
        ctx.step(s, 1e-3, p)
        out.append((s.numpy(), ctx.tess_counts()))
        ctx.close()
    assert out[0][1] == (0, 2) and out[1][1] == (0, 0)
    assert np.array_equal(out[0][0][0], out[1][0][0]) and np.array_equal(out[0][0][1], out[1][0][1])
