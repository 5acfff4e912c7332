"""The C-ABI libraries load on a machine without a GPU and export every
function their headers declare (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1410_3219_amd")

DECL = re.compile(r"^(?:int|void|const char\s*\*|rich_tess_ctx\s*\*)\s*\**\s*(rich_\w+)\s*\(",
                  re.M)


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(DECL.findall(text)))


@pytest.mark.parametrize("header,lib", [("rich.h", "librich.so"),
                                        ("rich_tess.h", "librichtess.so")])
def test_library_exports_every_declared_function(header, lib):
    names = declared(header)
    assert len(names) >= 10, names
    L = ctypes.CDLL(os.path.join(PKG, lib))
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_declared_entry_points_are_the_expected_set():
    names = set(declared("rich.h"))
    for must in ("rich_stage", "rich_stage_flags", "rich_cfl_dt", "rich_workspace_size",
                 "rich_stage_batch", "rich_batch_flags", "rich_batch_workspace_size",
                 "rich_step", "rich_step_batch", "rich_ctx_create", "rich_ctx_destroy",
                 "rich_ctx_set_mesh", "rich_ctx_mesh", "rich_strerror"):
        assert must in names


def test_strerror_without_gpu():
    L = ctypes.CDLL(os.path.join(PKG, "librich.so"))
    L.rich_strerror.restype = ctypes.c_char_p
    assert L.rich_strerror(0) == b"ok"
    assert b"mesh" in L.rich_strerror(-5)


def test_mesh_pack_is_a_bitwise_rearrangement():
    """rich_mesh_pack (host code, no GPU): the device records hold exactly the
    host stage's values, in the documented field order."""
    import numpy as np
    from paper_1410_3219_amd import inputs as I
    from paper_1410_3219_amd import rich as R
    from paper_1410_3219_amd import tess as T
    for bc in (0, 1):
        px, py = I.uniform_points(300, seed=3 + bc)
        m = T.rich_tess_build(px, py, (0.0, 0.0, 1.0, 1.0), bc)
        cells, edges = R.pack_mesh(m)
        cdt = np.dtype({"names": ["px", "py", "area", "sx", "sy", "pad"],
                        "formats": ["<f8"] * 6})
        edt = np.dtype({"names": ["fx", "fy", "len", "i", "j"],
                        "formats": ["<f8", "<f8", "<f8", "<i4", "<i4"]})
        assert cdt.itemsize == R.CELL_BYTES and edt.itemsize == R.EDGE_BYTES
        c = cells.view(cdt)
        e = edges.view(edt)
        assert c.shape[0] == m.n_cells and e.shape[0] == m.n_edges
        for f in ("px", "py", "area", "sx", "sy"):
            assert np.array_equal(c[f].view(np.uint64), getattr(m, f).view(np.uint64)), f
        assert (c["pad"] == 0).all()
        for f, g in (("fx", "e_fx"), ("fy", "e_fy"), ("len", "e_len"), ("i", "e_i"), ("j", "e_j")):
            a = e[f]
            b = getattr(m, g)
            assert np.array_equal(a.view(np.uint64) if a.dtype.itemsize == 8 else a,
                                  b.view(np.uint64) if b.dtype.itemsize == 8 else b), f
