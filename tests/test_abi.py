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
