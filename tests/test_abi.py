"""CPU checks of the C ABI: the in-tree library loads and exports every
function include/tr.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2010_04559_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2010_04559_amd import build
        build.build()
    return ctypes.CDLL(_lib.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("tr_setup", "tr_sweep", "tr_scatter", "tr_mg_vcycle", "tr_gmres_solve", "tr_adjoint_grad"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_2010_04559_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def test_last_error_is_callable_without_a_device(lib):
    lib.tr_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.tr_last_error(), bytes)


def test_setup_rejects_bad_arguments_before_touching_the_device(lib):
    from paper_2010_04559_amd import _lib
    L = _lib.load()
    p = _lib.TrProblem()
    p.dim = 4
    h = ctypes.c_void_p()
    assert L.tr_setup(ctypes.byref(p), ctypes.byref(h)) == _lib.TR_ERR_ARG
    assert b"dim" in L.tr_last_error()
    assert L.tr_setup(None, ctypes.byref(h)) == _lib.TR_ERR_ARG
