"""The OpenMP build of the oracle (used only to time it on all host cores)
gives the reference build's results bit for bit: each loop iteration writes
only its own cell or edge, with the same arithmetic."""
import os

import numpy as np
import pytest

import oracle as O
import parity_util as U


@pytest.mark.parametrize("name,k,riemann,pass2,integrator", [
    ("sedov", 40, 0, True, 0), ("wave", 36, 1, False, 0), ("kh", 30, 0, True, 0),
    ("sod", 33, 0, False, 1)])
def test_openmp_build_equals_reference_build(name, k, riemann, pass2, integrator):
    O.build()
    m, Qs, Qb, Xb, h, p = U.case(name, k=k, riemann=riemann, pass2=pass2,
                                 integrator=integrator)
    ref = O.stage(m, Qs, Qb, Xb, h, p, diag=True)
    assert O.threads() == 1
    with O.use_library(O.OMP_LIB_PATH):
        nthr = O.threads()
        par = O.stage(m, Qs, Qb, Xb, h, p, diag=True)
    assert par.status == ref.status == 0
    for a, b in ((ref.Q, par.Q), (ref.X, par.X), (ref.flux, par.flux), (ref.alpha, par.alpha)):
        assert np.array_equal(a, b)
    if (os.cpu_count() or 1) > 1:
        assert nthr > 1
