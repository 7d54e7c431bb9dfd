"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/msearch.h declares (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msearch.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("mesh_build", "propagate_vertices", "search_intersections", "last_error", "mesh_free",
              "search_workspace_size", "narrow_allpairs", "search_default_params", "mesh_info"):
        assert n in names, names


def test_library_exports_every_declared_symbol():
    import paper_2109_14814_amd as ms
    if not os.path.exists(ms.LIB_PATH):
        pytest.skip("libmsearch.so not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", ms.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for n in declared_functions():
        assert n in exported, n
    assert set(ms.EXPORTS) <= exported
    L = ctypes.CDLL(ms.LIB_PATH)
    for n in declared_functions():
        getattr(L, n)


def test_library_is_gfx950():
    import paper_2109_14814_amd as ms
    if not os.path.exists(ms.LIB_PATH):
        pytest.skip("libmsearch.so not built")
    data = open(ms.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_argument_errors_need_no_gpu():
    """Argument validation happens before any device call."""
    import paper_2109_14814_amd as ms
    if not os.path.exists(ms.LIB_PATH):
        pytest.skip("libmsearch.so not built")
    L = ms.lib()
    out = ctypes.c_void_p()
    assert L.mesh_build(None, -1, 3, 1, 0, None, None, None, ctypes.byref(out)) == ms.MS_E_ARG
    assert b"negative" in L.last_error()
    assert L.mesh_build(None, 4, 4, 1, 7, None, None, None, ctypes.byref(out)) == ms.MS_E_ARG
    p = ms.MapParams(0.01, 0.0, 0, 1)
    assert L.propagate_vertices(None, None, 10, ctypes.byref(p), None) == ms.MS_E_ARG
    assert L.mesh_free(None) == ms.MS_OK


def test_header_is_plain_c():
    """A C caller can include the header: it compiles as C99 with warnings as errors."""
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    subprocess.run(["gcc", "-fsyntax-only", "-x", "c", "-std=c99", "-Wall", "-Wextra", "-Werror", HEADER],
                   check=True)
