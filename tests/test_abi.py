"""Host-only checks of the C ABI: the library loads and exports every entry
point declared in include/*.h; defaults follow the paper's parameters.
No device work is done here."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
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
    assert "ls_plan_create" in names and "ls_solve" in names and "ls_fno_forward" in names
    assert len(names) >= 30
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
    assert o.sweep == 0 and o.level0 == 0


def test_status_strings_and_null_arguments():
    L = load()
    L.ls_status_str.restype = ctypes.c_char_p
    assert L.ls_status_str(0) == b"LS_OK" and L.ls_status_str(5) == b"LS_ESINGULAR"
    # argument validation happens before any device call
    L.ls_plan_create.restype = ctypes.c_int
    assert L.ls_plan_create(None, 64, ctypes.c_double(1 / 64), ctypes.c_double(1.0), None, None, None) == 1
    L.ls_plan_destroy.restype = ctypes.c_int
    assert L.ls_plan_destroy(None) == 0


def test_network_size_and_argument_checks():
    """The header's parameter count agrees with the library and with the
    flat layout of the seeded initial weights; bad sizes fail before any
    device work."""
    import ls_inputs as li
    L = load()
    L.ls_fno_param_count.restype = ctypes.c_size_t
    hdr = open(os.path.join(ROOT, "include", "ls_fno.h")).read()
    count = int(re.search(r"#define LS_FNO_PARAMS (\d+)", hdr).group(1))
    assert L.ls_fno_param_count() == count == sum(s for _, _, s in li.fno_param_sizes())
    L.ls_fno_create.restype = ctypes.c_int
    h = ctypes.c_void_p()
    assert L.ls_fno_create(ctypes.byref(h), 0, 64, None) == 1
    assert L.ls_fno_create(ctypes.byref(h), 2, 16, None) == 1
    L.ls_fno_destroy.restype = ctypes.c_int
    assert L.ls_fno_destroy(None) == 1
