"""The C-ABI library loads on a machine without a GPU and exports every entry point that
include/shellconv.h declares; the Python binding names the same set.  No compute calls."""
import ctypes
import os
import re

import pytest

import paper_2508_16635_amd as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shellconv.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sc_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for n in ("sc_plan_create", "sc_factor", "sc_step", "sc_jvp", "sc_newton_residual", "sc_set_base", "sc_newton"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(sc.LIB_PATH):
        pytest.skip("libshellconv.so not built")
    lib = ctypes.CDLL(sc.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_the_header():
    assert sorted(sc.exported_symbols()) == declared_symbols()


def test_binding_loads_and_types_every_entry_point():
    if not os.path.exists(sc.LIB_PATH):
        pytest.skip("libshellconv.so not built")
    lib = sc.load_library()
    for n in declared_symbols():
        fn = getattr(lib, n)
        assert fn.restype is not None


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        sc.load_library(str(tmp_path / "absent.so")) if sc._lib is None else _reload_missing(tmp_path)


def _reload_missing(tmp_path):
    saved = sc._lib
    sc._lib = None
    try:
        sc.load_library(str(tmp_path / "absent.so"))
    finally:
        sc._lib = saved


def test_plan_rejects_bad_mixed_solve():
    """Argument checks run before any device call, so this runs without a GPU."""
    if not os.path.exists(sc.LIB_PATH):
        pytest.skip("libshellconv.so not built")
    with pytest.raises(sc.ShellConvError) as ei:
        sc.Plan(8, 8, 2, 10, Ek=1e-3, Ra=50.0, mixed_solve=7)
    assert ei.value.code == 1
