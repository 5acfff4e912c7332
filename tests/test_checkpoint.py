"""Checkpoint and resume: the file round trip on the CPU, and on the GPU a run
stopped after k steps, saved, reloaded into a fresh step driver and continued
equals the uninterrupted run (bit for bit with host tessellation, to rounding
with device re-tessellation, whose first resumed step runs on the host-built
mesh of the same points)."""
import json

import numpy as np
import pytest

import parity_util as U
from paper_1410_3219_amd import checkpoint as CK
from paper_1410_3219_amd import inputs as I
from paper_1410_3219_amd import tess as T


def _setup(k=20):
    P = I.kelvin_helmholtz(k=k, seed=11)
    m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
    return P, m, P.state(m.area), np.stack([m.px, m.py])


def test_round_trip_on_cpu(tmp_path):
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _setup(9)
    s = R.DeviceState.from_host(Q, X, device="cpu")
    p = R.Params(gamma=P.gamma, riemann=1, limiter=2, gy=-0.5, integrator=1)
    f = tmp_path / "run.npz"
    CK.save(f, s, p, 0.125, 7, P.box, P.bc)
    s2, p2, t, step, box, bc = CK.load(f, device="cpu")
    assert np.array_equal(s2.Q.numpy(), Q) and np.array_equal(s2.X.numpy(), X)
    assert p2 == p and t == 0.125 and step == 7 and box == tuple(P.box) and bc == P.bc
    with np.load(f, allow_pickle=False) as z:
        assert set(z.files) == {"Q", "X", "meta"}


def test_rejects_foreign_or_malformed_files(tmp_path):
    f = tmp_path / "bad.npz"
    meta = {"format": "something-else"}
    np.savez(f, Q=np.zeros((4, 3)), X=np.zeros((2, 3)),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    with pytest.raises(ValueError):
        CK.load(f, device="cpu")
    meta = {"format": CK.FORMAT, "t": 0.0, "step": 0, "box": [0, 1, 0, 1], "bc": 0,
            "params": {}}
    np.savez(f, Q=np.zeros((4, 3)), X=np.zeros((2, 4)),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    with pytest.raises(ValueError):
        CK.load(f, device="cpu")


@pytest.mark.gpu
@pytest.mark.parametrize("device_tess", [False, True])
def test_resumed_run_equals_uninterrupted_run(tmp_path, device_tess):
    import torch
    from paper_1410_3219_amd import rich as R
    P, m, Q, X = _setup(24)
    p = R.Params(gamma=P.gamma)
    dts = [2e-3] * 8
    ctx = R.RichCtx(device_tess=device_tess)
    ctx.set_mesh(m)
    s = R.DeviceState.from_host(Q, X)
    for dt in dts[:3]:
        ctx.step(s, dt, p)
    f = tmp_path / "run.npz"
    CK.save(f, s, p, sum(dts[:3]), 3, P.box, P.bc)
    for dt in dts[3:]:
        ctx.step(s, dt, p)
    torch.cuda.synchronize()
    Qa, Xa = s.numpy()
    ctx.close()

    ctx2, s2, p2, t, step = CK.resume(f, device_tess=device_tess)
    assert step == 3 and p2 == p
    for dt in dts[step:]:
        ctx2.step(s2, dt, p2)
    torch.cuda.synchronize()
    Qb, Xb = s2.numpy()
    ctx2.close()
    if not device_tess:
        assert np.array_equal(Qa, Qb) and np.array_equal(Xa, Xb)
    else:
        # per conserved quantity, relative to its largest magnitude
        err = np.abs(Qb - Qa).max(axis=1) / np.abs(Qa).max(axis=1).clip(1e-300)
        assert err.max() < U.TOL, err
        assert np.abs(Xb - Xa).max() < U.TOL
