"""Area change rate of the cells (rich_area_rate, section 5 eq. areachange)
through the C-ABI: against the oracle's or_area_rate on the same mesh and
point velocities, and against central differences of device-rebuilt meshes
(the moved cells' areas), which it must match to second order."""
import numpy as np
import pytest

import oracle as O
from paper_1410_3219_amd import inputs as I
from paper_1410_3219_amd import tess as T

pytestmark = pytest.mark.gpu


def _case(name, k):
    if name == "sod":
        P = I.sod(k=k, seed=2)
    elif name == "wave":
        P = I.advected_wave(k=k, seed=3)
    elif name == "sedov":
        P = I.sedov(k=k, seed=4, lloyd_iters=1)
    elif name == "gresho":
        P = I.gresho(k=k, seed=5)
    else:
        P = I.kelvin_helmholtz(k=k, seed=6)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = I.sedov_state(P, m.area) if name == "sedov" else P.state(m.area)
    return P, m, Q, np.stack([m.px, m.py])


@pytest.mark.parametrize("name,k", [("sod", 21), ("wave", 26), ("sedov", 24), ("gresho", 20),
                                    ("kh", 19)])
@pytest.mark.parametrize("motion", [0, 1])
def test_area_rate_matches_oracle(name, k, motion):
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _case(name, k)
    op = O.Params(gamma=P.gamma, motion=motion)
    prim = O.primitives(m, Q, op)
    w = O.point_velocity(m, prim, op)
    ref = O.area_rate(m, w)
    dm = R.DeviceMesh.from_host(m)
    s = R.DeviceState.from_host(Q, X)
    ws = R.workspace(m.n_cells)
    ad = R.rich_area_rate(dm, s, R.Params(gamma=P.gamma, motion=motion), ws).cpu().numpy()
    assert R.rich_stage_flags(ws) == 0
    # scale: perimeter times the largest point speed
    scale = 4.0 * np.sqrt(m.area.max()) * max(np.abs(w).max(), 1e-300)
    err = np.abs(ad - ref).max() / scale
    print(f"\n{name} motion={motion} n={m.n_cells} adot err {err:.2e}")
    assert err < 1e-12, err
    if motion == 0:
        assert (ad == 0).all()


@pytest.mark.parametrize("name", ["sod", "wave"])
def test_area_rate_is_the_derivative_of_rebuilt_areas(name):
    """(A(x + e w) - A(x - e w)) / 2e with both meshes rebuilt on the device
    approaches adot at second order in e."""
    from paper_1410_3219_amd import rich as R
    import torch
    P, m, Q, X = _case(name, 24)
    p = R.Params(gamma=P.gamma, motion=1)
    dm = R.DeviceMesh.from_host(m)
    s = R.DeviceState.from_host(Q, X)
    ws = R.workspace(m.n_cells)
    ad = R.rich_area_rate(dm, s, p, ws).cpu().numpy()
    op = O.Params(gamma=P.gamma, motion=1)
    w = O.point_velocity(m, O.primitives(m, Q, op), op)
    h = 1.0 / 24
    e0 = 1e-3 * h / np.abs(w).max()
    errs = []
    for e in (e0, e0 / 2):
        areas = []
        for sgn in (1.0, -1.0):
            Xm = X + sgn * e * w
            if m.bc == 1:
                Xm = np.stack([np.mod(Xm[0], 1.0), np.mod(Xm[1], 1.0)])
            bufs = R.DeviceMeshBufs(m.n_cells, m.box, m.bc)
            tws = R.retess_workspace(m.n_cells)
            R.rich_retess(dm, torch.from_numpy(Xm).cuda(), bufs, tws)
            st, info = R.rich_retess_result(tws)
            assert st == 0, info
            areas.append(R.mesh_to_host(bufs.mesh(), info["n_edges"], info["n_csr"]).area)
        fd = (areas[0] - areas[1]) / (2 * e)
        errs.append(np.abs(fd - ad).max() / np.abs(ad).max())
    print(f"\n{name} central-difference error {errs}")
    assert errs[0] < 1e-3   # relative to the largest |adot|, small in a near-uniform flow
    assert 0.15 < errs[1] / errs[0] < 0.35, errs


def test_area_rate_invalid_arguments():
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _case("sod", 8)
    dm = R.DeviceMesh.from_host(m)
    s = R.DeviceState.from_host(Q, X)
    with pytest.raises(R.RichError) as e:
        R.rich_area_rate(dm, s, R.Params(gamma=P.gamma), R.workspace(m.n_cells)[:512])
    assert e.value.status == R.RICH_E_NOMEM
    with pytest.raises(R.RichError) as e:
        R.rich_area_rate(dm, s, R.Params(gamma=0.5), R.workspace(m.n_cells))
    assert e.value.status == R.RICH_E_INVAL
