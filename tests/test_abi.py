"""The C-ABI library loads and exports every entry point include/ada.h declares
(no device compute here), and the pure host functions behave."""
import ctypes
import os
import re

import pytest

from paper_2007_11208_amd import ada

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ada.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(ada_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_solver_entry_points():
    names = declared_functions()
    for must in ("ada_create", "ada_destroy", "ada_last_error", "ada_workspace_size", "ada_solve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(ada.LIB_PATH):
        pytest.skip("libada.so not built")
    lib = ctypes.CDLL(ada.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_workspace_query_and_defaults():
    if not os.path.exists(ada.LIB_PATH):
        pytest.skip("libada.so not built")
    o = ada.make_opts()
    assert o.struct_size == ctypes.sizeof(ada.Opts)
    assert o.rcond_threshold < 0 and o.want_berr == 1 and o.layout == 0
    assert ada.workspace_size(0, 1, o) == 0
    assert ada.workspace_size(4, 0, o) == 0
    s1 = ada.workspace_size(100, 1, o)
    s2 = ada.workspace_size(200, 1, o)
    s3 = ada.workspace_size(200, 8, o)
    assert 0 < s1 < s2 < s3
    # dense workspace covers the factor copy and the SVD's V: at least 2 n^2 doubles
    assert s2 >= 2 * 200 * 200 * 8
    # band layout of a huge system does not reserve dense n^2 storage
    ob = ada.make_opts(layout=ada.LAYOUT_BAND, kl_in=5, ku_in=5)
    sb = ada.workspace_size(1_000_000, 1, ob)
    assert 0 < sb < 2e9


def test_solve_rejects_bad_arguments_on_the_host():
    if not os.path.exists(ada.LIB_PATH):
        pytest.skip("libada.so not built")
    L = ada.lib()
    res = ada.Result()
    rc = L.ada_solve(None, 4, 1, None, 4, None, 4, None, 4, None, 0, None, ctypes.byref(res), None)
    assert rc == ada.ERR_ARG
    assert "ctx" in ada.last_error()
