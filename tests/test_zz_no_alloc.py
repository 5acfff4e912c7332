"""rich_stage_noalloc (the stage on the library's own scratch, for callers
that cannot allocate) through the C-ABI: two calls in a row, the second on a
smaller mesh, each equal bit for bit to rich_stage with a caller workspace
and to the oracle's stage within the parity bars; the flag word comes back
through flag_out; a mesh beyond the scratch is refused."""
import numpy as np
import pytest

import oracle as O
import parity_util as U

pytestmark = pytest.mark.gpu


def _noalloc_and_workspace(m, Qs, Qb, Xb, h, p):
    import torch
    from paper_1410_3219_amd import rich as R
    dm = R.DeviceMesh.from_host(m)
    src = R.DeviceState.from_host(Qs, Xb)
    base = R.DeviceState.from_host(Qb, Xb)
    a = R.DeviceState.empty_like(base)
    a.Q.fill_(float("nan"))
    a.X.fill_(float("nan"))
    flag = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    R.rich_stage_noalloc(dm, src, base, a, h, U.gpu_params(p), flag_out=flag)
    torch.cuda.synchronize()
    Qa, Xa = a.numpy()
    fa = int(flag.cpu()[0])
    b = R.DeviceState.empty_like(base)
    ws = R.workspace(m.n_cells)
    R.rich_stage(dm, src, base, b, h, U.gpu_params(p), ws)
    fb = R.rich_stage_flags(ws)
    Qb2, Xb2 = b.numpy()
    return Qa, Xa, fa, Qb2, Xb2, fb


def test_noalloc_stage_equals_workspace_stage_and_oracle():
    print("\nno-alloc stage: sod 45x45 then wave 23x23", flush=True)
    for name, k, kw in (("sod", 45, {"pass2": True}), ("wave", 23, {})):
        m, Qs, Qb, Xb, h, p = U.case(name, k=k, **kw)
        Qa, Xa, fa, Qw, Xw, fw = _noalloc_and_workspace(m, Qs, Qb, Xb, h, p)
        assert fa == 0 and fw == 0, (name, fa, fw)
        assert np.array_equal(Qa, Qw) and np.array_equal(Xa, Xw), name
        U.check_stage(m, Qs, Qb, Xb, h, p, Qa, Xa, label=f"no-alloc {name} {k}x{k}")


def test_noalloc_flag_and_size_limit():
    import torch
    from paper_1410_3219_amd import rich as R
    m, Qs, Qb, Xb, h, p = U.case("sod", k=20)
    Qb = Qb.copy()
    Qb[0, 5] = -1.0                                     # a cell with negative mass
    Qa, Xa, fa, Qw, Xw, fw = _noalloc_and_workspace(m, Qs, Qb, Xb, h, p)
    assert fa & R.FLAG_DOMAIN and fw & R.FLAG_DOMAIN
    assert np.array_equal(Qa, Qw, equal_nan=True)
    # a clean call afterwards clears the flag again
    m2, Qs2, Qb2, Xb2, h2, p2 = U.case("wave", k=12)
    Qa2, Xa2, fa2, Qw2, Xw2, fw2 = _noalloc_and_workspace(m2, Qs2, Qb2, Xb2, h2, p2)
    assert fa2 == 0 and np.array_equal(Qa2, Qw2)
