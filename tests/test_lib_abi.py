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


STRUCTS = {"ds_sphere": "Sphere", "ds_robot": "Robot", "ds_params": "Params",
           "ds_problem": "Problem", "ds_result": "Result", "ds_seed_result": "SeedResult",
           "ds_latency_stats": "LatencyStats"}


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes record of the binding has the size and field offsets the
    C compiler gives the header's struct (compiled here with gcc)."""
    import subprocess
    from paper_2410_16727_amd import dsopt
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dsopt.h"', 'int main(void) {']
    for cname, pyname in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in getattr(dsopt, pyname)._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {}
    for line in out:
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, pyname in STRUCTS.items():
        cls = getattr(dsopt, pyname)
        assert ctypes.sizeof(cls) == got[(cname, "size")], cname
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == got[(cname, field)], (cname, field)
