"""The parity metrics themselves, on the CPU.

The oracle's unmodified source built with fused multiply-adds (gcc -mfma
-ffp-contract=fast) rounds differently from the reference build, as the GPU
path does.  Two builds of one correct algorithm must pass both bars with a
wide margin; an error planted in the result of a cell far below the domain's
largest values must fail the per-cell bar even where the per-quantity bar,
which divides by the domain maximum, cannot see it."""
import numpy as np
import pytest

import oracle as O
import parity_util as U


@pytest.fixture(scope="module")
def fma_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("oracle_fma") / "liboracle_fma.so")
    return O.build_variant(open(O.SRC_PATH).read(), out,
                           fp_flags=("-mfma", "-ffp-contract=fast"))


CASES = [("sedov", 48, 0, False), ("sedov", 48, 1, True), ("sod", 40, 0, True),
         ("wave", 40, 0, False), ("kh", 36, 1, True)]


@pytest.mark.parametrize("name,k,riemann,pass2", CASES)
def test_fma_build_passes_both_bars_with_margin(fma_lib, name, k, riemann, pass2):
    m, Qs, Qb, Xb, h, p = U.case(name, k=k, riemann=riemann, pass2=pass2)
    ref = O.stage(m, Qs, Qb, Xb, h, p, diag=True)
    assert ref.status == 0
    with O.use_library(fma_lib):
        alt = O.stage(m, Qs, Qb, Xb, h, p)
    assert alt.status == 0
    differs = not np.array_equal(alt.Q, ref.Q)
    eq, ex = U.errors(m, alt.Q, alt.X, ref.Q, ref.X, Qb, p)
    ec, where = U.cell_errors(m, alt.Q, Qb, ref.Q, h, p, ref, Qs=Qs)
    print(f"\n{name} k={k}: builds differ={differs}, per-quantity {eq}, per-cell {ec}")
    assert (eq < 1e-2 * U.TOL).all() and (ec < 1e-2 * U.TOL).all(), (eq, ec, where)


def test_fma_build_differs_from_reference_build(fma_lib):
    """The FMA build is a genuinely different rounding of the same method
    (otherwise the test above shows nothing)."""
    m, Qs, Qb, Xb, h, p = U.case("kh", k=36, pass2=True)
    ref = O.stage(m, Qs, Qb, Xb, h, p)
    with O.use_library(fma_lib):
        alt = O.stage(m, Qs, Qb, Xb, h, p)
    assert not np.array_equal(alt.Q, ref.Q)


def test_per_cell_bar_sees_an_error_in_an_ambient_cell():
    """Point explosion on 48^2 cells: an ambient cell holds 1.5e-6 A of
    energy against the blast cell's 1, so a 1e-3 relative error in it is
    below 1e-12 of the domain-wide scale (on 512^2 cells the same holds for
    an error of 17%).  Only the per-cell bar catches it."""
    m, Qs, Qb, Xb, h, p = U.case("sedov", k=48)
    ref = O.stage(m, Qs, Qb, Xb, h, p, diag=True)
    assert ref.status == 0
    i = int(np.argmin(np.abs(ref.Q[3])))          # an ambient cell
    bad = ref.Q.copy()
    bad[3, i] *= 1.0 + 1e-3
    eq, ex = U.errors(m, bad, ref.X, ref.Q, ref.X, Qb, p)
    ec, where = U.cell_errors(m, bad, Qb, ref.Q, h, p, ref, Qs=Qs)
    assert eq[3] < U.TOL                           # invisible to the domain-wide bar
    assert ec[3] > 1e3 * U.TOL and where[3] == i, (ec, where, i)
    # the same error planted in momentum of a cell at rest is caught too
    bad = ref.Q.copy()
    bad[1, i] += 1e-3 * abs(ref.Q[0, i]) * 1e-3
    ec, _ = U.cell_errors(m, bad, Qb, ref.Q, h, p, ref, Qs=Qs)
    assert ec[1] > U.TOL, ec
