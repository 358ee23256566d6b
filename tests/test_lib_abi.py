"""The C-ABI library loads and exports every entry point declared in
include/dsopt.h (no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsopt.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ds_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["ds_plan_create", "ds_esdf_upload", "ds_optimize_seeds", "ds_get_best",
              "ds_cost", "ds_cost_grad", "ds_serve_submit", "ds_serve_poll"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2410_16727_amd import dsopt
    if not os.path.exists(dsopt.LIB_PATH):
        pytest.fail("libdsopt.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(dsopt.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(dsopt.EXPORTED) == set(declared())
    L = dsopt.load()
    assert L.ds_version() == 100
    assert isinstance(L.ds_last_error(), bytes)


def test_struct_sizes_match_header_layout():
    from paper_2410_16727_amd import dsopt
    assert ctypes.sizeof(dsopt.Sphere) == 20
    assert ctypes.sizeof(dsopt.Result) == 40
    assert ctypes.sizeof(dsopt.SeedResult) == 48
    assert ctypes.sizeof(dsopt.Problem) == 16 + 56 + 16
