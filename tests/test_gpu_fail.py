"""Failure handling forced from the host: a NaN in the state, a cell of the
mesh with a negative area, and a CSR entry naming an edge that does not
exist each make a stage report RICH_FLAG_DOMAIN (the kernels check every
index they take from the mesh, so nothing is read out of bounds); the step
driver then returns RICH_E_DOMAIN and leaves the state as it was, and in a
batch only the corrupted run is flagged while the others equal their clean
results bit for bit."""
import dataclasses

import numpy as np
import pytest

import parity_util as U

pytestmark = pytest.mark.gpu


def _corrupt(kind, m, Qs):
    Qs = Qs.copy()
    if kind == "nan_state":
        Qs[3, 7] = np.nan
    elif kind == "negative_area":
        area = m.area.copy()
        area[11] = -area[11]
        m = dataclasses.replace(m, area=area)
    elif kind == "edge_index":
        idx = m.idx.copy()
        k = int(m.off[5])
        idx[k] = 2 * (m.n_edges + 17) + (idx[k] & 1)   # an edge past the end
        m = dataclasses.replace(m, idx=idx)
    return m, Qs


@pytest.mark.parametrize("kind", ["nan_state", "negative_area", "edge_index"])
def test_stage_reports_corrupt_input(kind):
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("sod", k=20)
    _, _, clean = U.gpu_stage(m, Qs, Qb, Xb, h, p)
    assert clean == 0
    mc, Qc = _corrupt(kind, m, Qs)
    _, _, flags = U.gpu_stage(mc, Qc, Qb, Xb, h, p)
    assert flags & R.FLAG_DOMAIN, kind


@pytest.mark.parametrize("kind", ["nan_state", "negative_area", "edge_index"])
def test_batch_flags_only_the_corrupt_run(kind):
    import torch
    from paper_1410_3219_amd import rich as R
    cases = [U.case("sod", k=17), U.case("wave", k=23), U.case("kh", k=19, pass2=True)]

    def run(bad):
        meshes, srcs, bases, outs, hs, ps = [], [], [], [], [], []
        for r, (m, Qs, Qb, Xb, h, p) in enumerate(cases):
            if r == bad:
                m, Qs = _corrupt(kind, m, Qs)
            meshes.append(R.DeviceMesh.from_host(m))
            srcs.append(R.DeviceState.from_host(Qs, Xb))
            bases.append(R.DeviceState.from_host(Qb, Xb))
            outs.append(R.DeviceState.empty_like(bases[-1]))
            hs.append(h)
            ps.append(U.gpu_params(p))
        ws = R.batch_workspace([m.n_cells for m, *_ in cases])
        R.rich_stage_batch(meshes, srcs, bases, outs, hs, ps, ws)
        flags = R.rich_batch_flags(len(cases), ws)
        torch.cuda.synchronize()
        return [o.numpy() for o in outs], flags

    good, gflags = run(None)
    assert gflags == [0, 0, 0]
    res, flags = run(1)
    assert flags[1] & R.FLAG_DOMAIN and flags[0] == 0 and flags[2] == 0
    for r in (0, 2):
        assert np.array_equal(res[r][0], good[r][0]) and np.array_equal(res[r][1], good[r][1])


def test_step_with_nan_state_is_not_committed():
    import torch
    from paper_1410_3219_amd import rich as R
    from paper_1410_3219_amd import inputs as I
    from paper_1410_3219_amd import tess as T
    P = I.sod(k=16, seed=3)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    Q = P.state(m.area)
    Q[0, 9] = np.nan
    X = np.stack([m.px, m.py])
    ctx = R.RichCtx()
    ctx.set_mesh(m)
    s = R.DeviceState.from_host(Q, X)
    with pytest.raises(R.RichError) as e:
        ctx.step(s, 1e-3, R.Params(gamma=P.gamma))
    assert e.value.status == R.RICH_E_DOMAIN
    torch.cuda.synchronize()
    Qa, Xa = s.numpy()
    assert np.array_equal(Qa, Q, equal_nan=True) and np.array_equal(Xa, X)
    ctx.close()
