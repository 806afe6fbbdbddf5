"""Host-only checks of the C ABI: the library loads and exports every entry
point declared in include/ls.h; defaults follow the paper's parameters.
No device work is done here."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ls.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[A-Za-z_0-9]+)\s*\(", src)))


def load():
    from paper_1602_07652_amd.build import lib_path
    path = lib_path()
    if not os.path.exists(path):
        from paper_1602_07652_amd.build import build
        build(verbose=False)
    return ctypes.CDLL(path)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "ls_plan_create" in names and "ls_solve" in names and len(names) >= 18
    L = load()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_defaults_follow_the_paper():
    from paper_1602_07652_amd import default_options
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    o = default_options()
    assert o.inner_tol == gold["inner_tol"]["value"]
    assert o.ext == gold["extension_points"]["value"]
    assert o.precond == 0 and o.max_batch == 1 and o.inner_fixed_iters == 0


def test_status_strings_and_null_arguments():
    L = load()
    L.ls_status_str.restype = ctypes.c_char_p
    assert L.ls_status_str(0) == b"LS_OK" and L.ls_status_str(5) == b"LS_ESINGULAR"
    # argument validation happens before any device call
    L.ls_plan_create.restype = ctypes.c_int
    assert L.ls_plan_create(None, 64, ctypes.c_double(1 / 64), ctypes.c_double(1.0), None, None, None) == 1
    L.ls_plan_destroy.restype = ctypes.c_int
    assert L.ls_plan_destroy(None) == 0
