"""HIP stage against the oracle, element by element, through the C-ABI.

Every case feeds both sides the same seeded mesh and state; the bar is
1e-12 relative per conserved quantity (see parity_util).  Sizes span several
256-cell tiles and a ragged last tile."""
import numpy as np
import pytest

import oracle as O
import parity_util as U
from paper_1410_3219_amd import inputs as I
from paper_1410_3219_amd import tess as T

pytestmark = pytest.mark.gpu


def _run(name, **kw):
    m, Qs, Qb, Xb, h, p = U.case(name, **kw)
    ref = O.stage(m, Qs, Qb, Xb, h, p, diag=True)
    assert ref.status == 0
    Qg, Xg, flags = U.gpu_stage(m, Qs, Qb, Xb, h, p)
    assert flags == 0
    U.check_stage(m, Qs, Qb, Xb, h, p, Qg, Xg, ref=ref, label=f"{name} {kw}")
    return m


@pytest.mark.parametrize("name,k", [("sod", 24), ("sod", 37), ("sod_angle", 30), ("wave", 33),
                                    ("acoustic", 20), ("sedov", 28), ("kh", 26),
                                    ("gresho", 30)])
@pytest.mark.parametrize("pass2", [False, True])
def test_stage_hllc(name, k, pass2):
    _run(name, k=k, pass2=pass2)


@pytest.mark.parametrize("name,pass2", [("sod", False), ("sod", True), ("kh", True),
                                        ("sedov", False)])
def test_stage_external_acceleration(name, pass2):
    _run(name, k=29, pass2=pass2, g=(0.4, -1.1))


@pytest.mark.parametrize("name,riemann", [("sod", 0), ("wave", 0), ("sedov", 0), ("kh", 0),
                                          ("gresho", 0), ("sod", 1)])
def test_stage_extrapolated_fluxes(name, riemann):
    """The extrapolated-fluxes stage (face states advanced half a step)."""
    _run(name, k=27, riemann=riemann, integrator=1)


@pytest.mark.parametrize("name", ["sod", "wave", "sedov"])
def test_stage_exact_riemann(name):
    _run(name, k=27, riemann=1)
    _run(name, k=27, riemann=1, pass2=True)


@pytest.mark.parametrize("limiter", [1, 2, 3, 4])
@pytest.mark.parametrize("motion", [0, 1])
def test_stage_limiters_and_motion(limiter, motion):
    if limiter == 3:
        # unlimited reconstruction is only sound on smooth data
        _run("acoustic", k=25, limiter=limiter, motion=motion)
        _run("gresho", k=23, limiter=limiter, motion=motion, pass2=True)
        return
    _run("sod_angle", k=25, limiter=limiter, motion=motion)
    _run("kh", k=23, limiter=limiter, motion=motion, pass2=True)


@pytest.mark.parametrize("name,k", [("sod", 1), ("sod", 2), ("wave", 1), ("wave", 2),
                                    ("kh", 3), ("sod", 16)])
def test_stage_tiny_and_exact_tile(name, k):
    # one cell, a few cells, and exactly one full 256-cell tile
    _run(name, k=k)


@pytest.mark.parametrize("bc", [0, 1])
def test_stage_cells_in_random_order(bc):
    """20 000 uniform-random points in random (not Hilbert) order: most of a
    tile's neighbours lie in other tiles, so tiles own more edges than the
    LDS slots hold and touch more foreign edges than the LDS list holds;
    those fluxes are recomputed in the gather.  Both stages, walls and a
    periodic box."""
    px, py = I.uniform_points(20000, seed=5 + bc, sort=False)
    box = (0.0, 0.0, 1.0, 1.0)
    m = T.rich_tess_build(px, py, box, bc)
    rho = np.where(px < 0.5, 1.0, 0.125)
    pr = np.where(px < 0.5, 1.0, 0.1)
    Q = I.conserved(rho, 0.2, -0.1, pr, m.area, 5.0 / 3.0)
    X = np.stack([m.px, m.py])
    p = O.Params(gamma=5.0 / 3.0)
    dt, st = O.cfl_dt(m, Q, p)
    assert st == 0
    ref = O.stage(m, Q, Q, X, 0.5 * dt, p, diag=True)
    assert ref.status == 0
    Qg, Xg, flags = U.gpu_stage(m, Q, Q, X, 0.5 * dt, p)
    assert flags == 0
    U.check_stage(m, Q, Q, X, 0.5 * dt, p, Qg, Xg, ref=ref, label=f"random order bc={bc} stage 1")
    mh = T.rich_tess_build(ref.X[0], ref.X[1], box, bc)
    ref2 = O.stage(mh, ref.Q, Q, X, dt, p, diag=True)
    assert ref2.status == 0
    Qg2, Xg2, flags = U.gpu_stage(mh, ref.Q, Q, X, dt, p)
    assert flags == 0
    U.check_stage(mh, ref.Q, Q, X, dt, p, Qg2, Xg2, ref=ref2,
                  label=f"random order bc={bc} stage 2")


def test_deterministic_repeat():
    m, Qs, Qb, Xb, h, p = U.case("sedov", k=40)
    outs = U.gpu_stage(m, Qs, Qb, Xb, h, p, repeat=3)
    for Q, X, f in outs[1:]:
        assert np.array_equal(Q, outs[0][0]) and np.array_equal(X, outs[0][1])


def test_cfl_dt():
    import torch
    from paper_1410_3219_amd import rich as R
    for name in ("sod", "wave", "sedov", "kh"):
        m, Qs, Qb, Xb, h, p = U.case(name, k=30)
        dt_ref, st = O.cfl_dt(m, Qs, p)
        dm = R.DeviceMesh.from_host(m)
        s = R.DeviceState.from_host(Qs, Xb)
        ws = R.workspace(m.n_cells)
        dt = R.rich_cfl_dt(dm, s, U.gpu_params(p), ws)
        assert abs(dt - dt_ref) <= 1e-13 * dt_ref, (name, dt, dt_ref)


@pytest.mark.parametrize("k", [1, 2100])
def test_cfl_dt_grid_sizes(k):
    """A single cell, and 4 410 000 cells: more cells than one pass of the
    bounded reduction grid (16 384 blocks of 256) covers, so blocks stride
    over the cells."""
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("wave", k=k)
    dt_ref, st = O.cfl_dt(m, Qs, p)
    assert st == 0
    dm = R.DeviceMesh.from_host(m)
    s = R.DeviceState.from_host(Qs, Xb)
    dt = R.rich_cfl_dt(dm, s, U.gpu_params(p), R.workspace(m.n_cells))
    assert abs(dt - dt_ref) <= 1e-13 * dt_ref, (k, dt, dt_ref)


def test_domain_error_flag():
    # negative mass in one cell: the stage reports it and still writes
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("sod", k=20)
    Qb = Qb.copy()
    Qb[0, 5] = -1.0
    Qg, Xg, flags = U.gpu_stage(m, Qs, Qb, Xb, h, p)
    assert flags & R.FLAG_DOMAIN
    ref = O.stage(m, Qs, Qb, Xb, h, p)
    assert ref.status == -4


def test_invalid_arguments_rejected():
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("sod", k=8)
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    out = R.DeviceState.empty_like(src)
    ws = R.workspace(m.n_cells)
    with pytest.raises(R.RichError) as e:
        R.rich_stage(dm, src, src, out, float("nan"), U.gpu_params(p), ws)
    assert e.value.status == R.RICH_E_INVAL
    with pytest.raises(R.RichError) as e:
        R.rich_stage(dm, src, src, src, h, U.gpu_params(p), ws)   # out aliases src
    assert e.value.status == R.RICH_E_INVAL
    small = ws[: ws.numel() // 2]
    with pytest.raises(R.RichError) as e:
        R.rich_stage(dm, src, src, out, h, U.gpu_params(p), small)
    assert e.value.status == R.RICH_E_NOMEM


@pytest.mark.parametrize("integrator", [0, 1])
def test_full_size_wave_stage(integrator):
    """The benchmark workload at full size (2048^2 = 4 194 304 cells,
    12 582 912 edges, periodic, moving mesh, HLLC), compared with the oracle
    on every cell: stage 1 of the time-centred step in the launch
    configuration the benchmark times, and the one full-step stage of the
    extrapolated-fluxes integrator."""
    P = I.advected_wave(k=2048, seed=3)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    assert m.n_cells == 2048 * 2048 and m.n_edges == 3 * m.n_cells
    Q = P.state(m.area)
    X = np.stack([m.px, m.py])
    p = O.Params(gamma=P.gamma, integrator=integrator)
    dt, st = O.cfl_dt(m, Q, p)
    assert st == 0
    h = 0.5 * dt if integrator == 0 else dt
    ref = O.stage(m, Q, Q, X, h, p, diag=True)
    assert ref.status == 0
    Qg, Xg, flags = U.gpu_stage(m, Q, Q, X, h, p)
    assert flags == 0
    U.check_stage(m, Q, Q, X, h, p, Qg, Xg, ref=ref,
                  label=f"full-size wave, integrator {integrator}")


def test_full_size_point_explosion_step():
    """The point-explosion configuration at full size (262 144 uniform-random
    points Lloyd-relaxed 5 times, walls, E = 1 in the centre cell, exact and
    HLLC solvers): both stages of a time-centred step, each compared with
    the oracle on every cell from the same inputs."""
    P = I.sedov(k=512, seed=2, lloyd_iters=5)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = I.sedov_state(P, m.area)
    X = np.stack([m.px, m.py])
    for riemann in (0, 1):
        p = O.Params(gamma=P.gamma, riemann=riemann)
        dt, st = O.cfl_dt(m, Q, p)
        assert st == 0
        ref1 = O.stage(m, Q, Q, X, 0.5 * dt, p, diag=True)
        assert ref1.status == 0
        Qh, Xh, flags = U.gpu_stage(m, Q, Q, X, 0.5 * dt, p)
        assert flags == 0
        U.check_stage(m, Q, Q, X, 0.5 * dt, p, Qh, Xh, ref=ref1,
                      label=f"sedov 512^2 riemann={riemann} stage 1")
        mh = T.rich_tess_build(Xh[0], Xh[1], m.box, m.bc)
        ref2 = O.stage(mh, Qh, Q, X, dt, p, diag=True)
        assert ref2.status == 0
        Qn, Xn, flags = U.gpu_stage(mh, Qh, Q, X, dt, p)
        assert flags == 0
        U.check_stage(mh, Qh, Q, X, dt, p, Qn, Xn, ref=ref2,
                      label=f"sedov 512^2 riemann={riemann} stage 2")


def _gpu_stage_accel(m, Qs, Qb, Xb, h, p, a):
    import torch
    from paper_1410_3219_amd import rich as R
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    base = R.DeviceState.from_host(Qb, Xb)
    out = R.DeviceState.empty_like(base)
    ws = R.workspace(m.n_cells)
    R.rich_stage_accel(dm, src, base, out, h, U.gpu_params(p), torch.from_numpy(a).cuda(), ws)
    flags = R.rich_stage_flags(ws)
    torch.cuda.synchronize()
    return (*out.numpy(), flags)


@pytest.mark.parametrize("name,k,pass2,riemann", [("sod", 21, False, 0), ("kh", 24, True, 0),
                                                  ("wave", 19, False, 1), ("sedov", 23, True, 0)])
def test_stage_acceleration_field(name, k, pass2, riemann):
    """A per-cell external acceleration added to a uniform one (section 2.3
    source term): rich_stage_accel against the oracle's stage with the same
    field, walls and periodic boxes, both stages, both solvers."""
    m, Qs, Qb, Xb, h, p = U.case(name, k=k, riemann=riemann, pass2=pass2, g=(0.05, -0.3))
    rng = np.random.default_rng(k)
    a = np.stack([0.8 * np.sin(2 * np.pi * m.px) + rng.uniform(-0.1, 0.1, m.n_cells),
                  -0.5 * np.cos(2 * np.pi * m.py)])
    ref = O.stage_accel(m, Qs, Qb, Xb, h, p, a)
    assert ref.status == 0
    Qg, Xg, flags = _gpu_stage_accel(m, Qs, Qb, Xb, h, p, a)
    assert flags == 0
    U.check_stage(m, Qs, Qb, Xb, h, p, Qg, Xg, ref=ref, accel=a, label=f"accel field {name}")
    # the field adds h M_src a to the momentum of the stage without it
    Q0, _, _ = U.gpu_stage(m, Qs, Qb, Xb, h, p)
    for q in (1, 2):
        want = h * Qs[0] * a[q - 1]
        tol = 1e-9 * np.abs(want).max() + 1e-14 * np.abs(Qg[q]).max()
        assert np.abs((Qg[q] - Q0[q]) - want).max() < tol, q


def test_stage_field_view_on_side_stream_equals_contiguous_field():
    """A non-contiguous (2, n) field passed with a stream other than torch's
    current one: the binding's contiguous copy is ordered before the stage on
    that stream and kept alive for it; the result equals the contiguous
    field's bit for bit."""
    import torch
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("kh", k=22, pass2=True, g=(0.1, -0.2))
    a = np.stack([0.3 * np.sin(2 * np.pi * m.py), -0.4 * np.cos(2 * np.pi * m.px)])
    Qc, Xc, fc = _gpu_stage_accel(m, Qs, Qb, Xb, h, p, a)
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    base = R.DeviceState.from_host(Qb, Xb)
    out = R.DeviceState.empty_like(base)
    ws = R.workspace(m.n_cells)
    view = torch.from_numpy(np.ascontiguousarray(a.T)).cuda().T   # (2, n), strides (1, 2)
    assert not view.is_contiguous()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    R.rich_stage_accel(dm, src, base, out, h, U.gpu_params(p), view, ws, stream=side)
    del view
    side.synchronize()
    Qv, Xv = out.numpy()
    assert fc == 0 and R.rich_stage_flags(ws) == 0
    assert np.array_equal(Qv, Qc) and np.array_equal(Xv, Xc)


def test_stage_constant_field_equals_uniform_acceleration():
    """A field equal to (cx, cy) everywhere gives the stage of the uniform
    acceleration (cx, cy) bit for bit; a missing field is rejected."""
    import ctypes as C
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("kh", k=20, g=(0.3, -0.7))
    Qu, Xu, fu = U.gpu_stage(m, Qs, Qb, Xb, h, p)
    p0 = O.Params(gamma=p.gamma, riemann=p.riemann, limiter=p.limiter, motion=p.motion)
    a = np.stack([np.full(m.n_cells, 0.3), np.full(m.n_cells, -0.7)])
    Qa, Xa, fa = _gpu_stage_accel(m, Qs, Qb, Xb, h, p0, a)
    assert fu == 0 and fa == 0
    assert np.array_equal(Qa, Qu) and np.array_equal(Xa, Xu)
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    out = R.DeviceState.empty_like(src)
    ws = R.workspace(m.n_cells)
    st = R.lib().rich_stage_accel(C.byref(dm.c()), C.byref(src.c()), C.byref(src.c()),
                                  C.byref(out.c()), float(h), C.byref(U.gpu_params(p).c()),
                                  None, None, C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == R.RICH_E_INVAL
