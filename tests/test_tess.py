"""Host input stage (section 2.1): Delaunay by point insertion with exact
predicates, Voronoi read off the triangulation, ghost points for walls and
periodic boxes.  Pinned by brute force and by geometric identities."""
import math

import numpy as np
import pytest

from paper_1410_3219_amd import inputs as I

BOX = (0.0, 0.0, 1.0, 1.0)


def circumcentre(ax, ay, bx, by, cx, cy):
    d = 2 * ((bx - ax) * (cy - ay) - (by - ay) * (cx - ax))
    b2 = (bx - ax) ** 2 + (by - ay) ** 2
    c2 = (cx - ax) ** 2 + (cy - ay) ** 2
    return ax + ((cy - ay) * b2 - (by - ay) * c2) / d, ay + ((bx - ax) * c2 - (cx - ax) * b2) / d


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 7, 60, 400])
def test_empty_circumcircle_brute_force(tess_mod, bc, n):
    px, py = I.uniform_points(n, seed=10 + n, box=BOX)
    x, y, gs, tri = tess_mod.rich_tess_triangles(px, py, BOX, bc)
    assert tri.shape[0] > 0
    for a, b, c in tri:
        d = (x[b] - x[a]) * (y[c] - y[a]) - (y[b] - y[a]) * (x[c] - x[a])
        assert d > 0  # counter-clockwise, non-degenerate
        ux, uy = circumcentre(x[a], y[a], x[b], y[b], x[c], y[c])
        r2 = (x[a] - ux) ** 2 + (y[a] - uy) ** 2
        dd = (x - ux) ** 2 + (y - uy) ** 2
        dd[[a, b, c]] = np.inf
        assert not (dd < r2 * (1 - 1e-9)).any()


def mesh_checks(m, n, box, bc):
    Lx, Ly = box[2] - box[0], box[3] - box[1]
    # cells tile the box
    assert abs(m.area.sum() - Lx * Ly) < 1e-13 * Lx * Ly
    assert (m.area > 0).all()
    # closed edge-normal sums: sum_j L_ij n_ij = 0 per cell
    cell = m.nb_cell()
    code = m.nb_code()
    sx = np.zeros(m.n_edges)
    sy = np.zeros(m.n_edges)
    per = (code >= 1) & (code <= 8)
    k = np.where(code <= 4, code - 1, code)
    sx[per] = (k[per] // 3 - 1) * Lx
    sy[per] = (k[per] % 3 - 1) * Ly
    wall = code >= 9
    rjx = m.px[cell] + sx
    rjy = m.py[cell] + sy
    ii = m.e_i
    rjx[wall] = np.where(code[wall] == 9, 2 * box[0] - m.px[ii[wall]],
                         np.where(code[wall] == 10, 2 * box[2] - m.px[ii[wall]], m.px[ii[wall]]))
    rjy[wall] = np.where(code[wall] == 11, 2 * box[1] - m.py[ii[wall]],
                         np.where(code[wall] == 12, 2 * box[3] - m.py[ii[wall]], m.py[ii[wall]]))
    dx, dy = rjx - m.px[ii], rjy - m.py[ii]
    d = np.hypot(dx, dy)
    nx, ny = dx / d, dy / d
    # the edge centre lies on the perpendicular bisector of the two points
    cx = m.e_fx - 0.5 * (m.px[ii] + rjx)
    cy = m.e_fy - 0.5 * (m.py[ii] + rjy)
    assert np.max(np.abs(cx * nx + cy * ny)) < 1e-12 * max(Lx, Ly)
    accx = np.zeros(n)
    accy = np.zeros(n)
    for c in range(n):
        for k_ in range(m.off[c], m.off[c + 1]):
            e, side = m.idx[k_] >> 1, m.idx[k_] & 1
            s = -1.0 if side else 1.0
            accx[c] += s * m.e_len[e] * nx[e]
            accy[c] += s * m.e_len[e] * ny[e]
    scale = np.sqrt(m.area)
    assert np.max(np.abs(accx) / scale) < 1e-12
    assert np.max(np.abs(accy) / scale) < 1e-12
    # CSR consistency: every non-wall edge appears once per side
    cnt = np.zeros(m.n_edges, dtype=int)
    for c in range(n):
        for k_ in range(m.off[c], m.off[c + 1]):
            e, side = m.idx[k_] >> 1, m.idx[k_] & 1
            owner = m.e_i[e] if side == 0 else cell[e]
            assert owner == c
            cnt[e] += 1
    assert (cnt[~wall] == 2).all() and (cnt[wall] == 1).all()
    # edges sorted by owner, eoff consistent
    assert (np.diff(m.e_i) >= 0).all()
    for c in range(n):
        assert (m.e_i[m.eoff[c]:m.eoff[c + 1]] == c).all()
    # centroid = area-weighted mean of the polygon: check via sum A s = box centroid
    if bc == 0:
        cxm = (m.area * m.sx).sum() / m.area.sum()
        cym = (m.area * m.sy).sum() / m.area.sum()
        assert abs(cxm - 0.5 * (box[0] + box[2])) < 1e-12
        assert abs(cym - 0.5 * (box[1] + box[3])) < 1e-12


@pytest.mark.parametrize("bc", [0, 1])
def test_mesh_identities_random(tess_mod, bc):
    n = 600
    px, py = I.uniform_points(n, seed=3, box=BOX)
    m = tess_mod.rich_tess_build(px, py, BOX, bc)
    mesh_checks(m, n, BOX, bc)
    if bc == 1:
        # Euler's formula on the torus with degree-3 Voronoi vertices: E = 3N
        assert m.n_edges == 3 * n


def test_points_near_walls_large_random(tess_mod):
    """151 321 uniform-random points with walls: many points lie within
    1e-5 of a wall, so the triangulation joins cells to the mirror images of
    other cells across co-circular trapezoids.  Those zero-length edges are
    dropped; the mesh closes (every cell's sum of L n over its CSR entries
    vanishes, areas tile the box) and every wall edge is a cell's own
    mirror."""
    px, py = I.uniform_points(389 * 389, seed=14, box=BOX)
    m = tess_mod.rich_tess_build(px, py, BOX, 0)
    n = px.shape[0]
    assert abs(m.area.sum() - 1.0) < 1e-12
    code = (m.e_j.view(np.uint32) >> 28).astype(np.int64)
    cell = (m.e_j & 0x0FFFFFFF).astype(np.int64)
    wall = code >= 9
    assert (cell[wall] == m.e_i[wall]).all()
    # outward unit normals from e_i towards its neighbour (mirror for walls)
    rjx, rjy = m.px[cell].copy(), m.py[cell].copy()
    rjx[code == 9] = -m.px[m.e_i[code == 9]]
    rjx[code == 10] = 2.0 - m.px[m.e_i[code == 10]]
    rjy[code == 11] = -m.py[m.e_i[code == 11]]
    rjy[code == 12] = 2.0 - m.py[m.e_i[code == 12]]
    dx, dy = rjx - m.px[m.e_i], rjy - m.py[m.e_i]
    d = np.hypot(dx, dy)
    e = m.idx >> 1
    sgn = np.where(m.idx & 1, -1.0, 1.0)
    owner = np.repeat(np.arange(n), np.diff(m.off))
    ax = np.zeros(n)
    ay = np.zeros(n)
    np.add.at(ax, owner, sgn * m.e_len[e] * dx[e] / d[e])
    np.add.at(ay, owner, sgn * m.e_len[e] * dy[e] / d[e])
    assert np.max(np.hypot(ax, ay) / np.sqrt(m.area)) < 1e-9


@pytest.mark.parametrize("bc", [0, 1])
def test_mesh_identities_jittered_rect_box(tess_mod, bc):
    box = (-0.5, -1.0, 1.5, 0.25)
    px, py = I.jittered_lattice(20, seed=4, jitter=0.2, box=box, ky=13)
    m = tess_mod.rich_tess_build(px, py, box, bc)
    mesh_checks(m, px.shape[0], box, bc)


@pytest.mark.parametrize("bc", [0, 1])
def test_degenerate_square_lattice(tess_mod, bc):
    # every quadruple of neighbouring points is co-circular: the zero-length
    # Voronoi edges are dropped and the cells are exact squares
    k = 12
    px, py = I.lattice(k, BOX)
    m = tess_mod.rich_tess_build(px, py, BOX, bc)
    h = 1.0 / k
    assert np.allclose(m.area, h * h, rtol=1e-13, atol=0)
    assert np.allclose(m.sx, m.px, atol=1e-15) and np.allclose(m.sy, m.py, atol=1e-15)
    assert np.allclose(m.e_len, h, rtol=1e-12)
    assert m.diag["n_exact"] > 0
    nint = 2 * k * (k - 1)
    assert m.n_edges == (nint + 4 * k if bc == 0 else 2 * k * k)
    mesh_checks(m, k * k, BOX, bc)


def test_tiny_meshes(tess_mod):
    for bc in (0, 1):
        for n in (1, 2, 3):
            px, py = I.uniform_points(n, seed=20 + n, box=BOX)
            m = tess_mod.rich_tess_build(px, py, BOX, bc)
            assert abs(m.area.sum() - 1.0) < 1e-14


def test_invalid_inputs(tess_mod):
    with pytest.raises(tess_mod.TessError) as e:
        tess_mod.rich_tess_build(np.array([0.5, 0.5]), np.array([0.5, 0.5]), BOX, 0)
    assert e.value.status == -5  # duplicate points
    with pytest.raises(tess_mod.TessError) as e:
        tess_mod.rich_tess_build(np.array([1.5]), np.array([0.5]), BOX, 0)
    assert e.value.status == -1  # outside a walled box
    with pytest.raises(tess_mod.TessError):
        tess_mod.rich_tess_build(np.array([np.nan]), np.array([0.5]), BOX, 1)


def test_periodic_wrap(tess_mod):
    px, py = I.uniform_points(50, seed=8, box=BOX)
    m1 = tess_mod.rich_tess_build(px, py, BOX, 1)
    m2 = tess_mod.rich_tess_build(px + 3.0, py - 1.0, BOX, 1)
    assert np.allclose(m1.area, m2.area, rtol=1e-12)


def test_predicates_exact(tess_mod):
    # nearly collinear / co-circular inputs where plain evaluation fails
    a = [0.5, 0.5]
    b = [12.0, 12.0]
    x = 24.0
    for k in range(1, 20):
        x = np.nextafter(x, 25.0)
        c = [x, 24.0]  # just right of (below) the line y = x
        assert tess_mod.rich_tess_orient2d(a, b, c) == -1
        assert tess_mod.rich_tess_orient2d(b, a, c) == 1
    assert tess_mod.rich_tess_orient2d(a, b, [24.0, 24.0]) == 0
    # small perturbations of a near-collinear triple around 0.5: plain
    # evaluation is unreliable, the exact one agrees with rational arithmetic
    from fractions import Fraction as Fr
    for i in range(64):
        for j in range(64):
            p = [0.5 + i * 2.0 ** -53, 0.5 + j * 2.0 ** -53]
            q, r = [12.0, 12.0], [24.0, 24.0]
            det = (Fr(q[0]) - Fr(p[0])) * (Fr(r[1]) - Fr(p[1])) - \
                  (Fr(q[1]) - Fr(p[1])) * (Fr(r[0]) - Fr(p[0]))
            want = (det > 0) - (det < 0)
            assert tess_mod.rich_tess_orient2d(p, q, r) == want
    # co-circular unit-circle points and a point nudged inside / outside
    pts = [[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]]
    assert tess_mod.rich_tess_incircle(*pts, [0.0, -1.0]) == 0
    assert tess_mod.rich_tess_incircle(*pts, [0.0, np.nextafter(-1.0, 0.0)]) == 1
    assert tess_mod.rich_tess_incircle(*pts, [0.0, np.nextafter(-1.0, -2.0)]) == -1
    # scaled lattice quad: exactly co-circular
    h = 0.1
    assert tess_mod.rich_tess_incircle([0, 0], [h, 0], [h, h], [0, h]) == 0


def test_hilbert_order_is_permutation(tess_mod):
    px, py = I.uniform_points(1000, seed=1, box=BOX, sort=False)
    perm = tess_mod.rich_tess_hilbert_order(px, py, BOX)
    assert sorted(perm.tolist()) == list(range(1000))
    # consecutive points along the curve are close on average
    d = np.hypot(np.diff(px[perm]), np.diff(py[perm]))
    assert d.mean() < 3.0 / math.sqrt(1000)


def test_lloyd_moves_points_to_centroids(tess_mod):
    px, py = I.uniform_points(300, seed=2, box=BOX)
    qx, qy = tess_mod.rich_tess_lloyd(px, py, BOX, 0, 3)
    m = tess_mod.rich_tess_build(qx, qy, BOX, 0)
    m0 = tess_mod.rich_tess_build(px, py, BOX, 0)
    off0 = np.hypot(m0.sx - m0.px, m0.sy - m0.py).mean()
    off3 = np.hypot(m.sx - m.px, m.sy - m.py).mean()
    assert off3 < 0.5 * off0
