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


# ------------------------------------------------------------ failure paths
# Every check below happens in tr_setup / tr_workspace_bytes before any
# device call, so the CPU test run exercises them through the C ABI.

def _setup_rc(prob):
    from paper_2010_04559_amd import _lib
    from paper_2010_04559_amd.transport import problem_struct
    L = _lib.load()
    p, keep = problem_struct(prob)
    h = ctypes.c_void_p()
    rc = L.tr_setup(ctypes.byref(p), ctypes.byref(h))
    assert not h.value, "no handle may be returned on failure"
    return rc, L.tr_last_error().decode()


def _small():
    from paper_2010_04559_amd import inputs
    return inputs.small_problem(dim=3, n=4, level=1, order=4)


@pytest.mark.parametrize("bad", [float("nan"), 0.0, -1.0, float("inf")])
def test_setup_rejects_bad_sigma_t(bad):
    from paper_2010_04559_amd import _lib
    prob = _small()
    st = prob.sigma_t.copy()
    st[5] = bad
    rc, msg = _setup_rc(prob.with_sigma(st, prob.sigma_s))
    assert rc == _lib.TR_ERR_ARG and "sigma_t" in msg


@pytest.mark.parametrize("bad", [float("nan"), -0.5])
def test_setup_rejects_bad_sigma_s(bad):
    from paper_2010_04559_amd import _lib
    prob = _small()
    ss = prob.sigma_s.copy()
    ss[3] = bad
    rc, msg = _setup_rc(prob.with_sigma(prob.sigma_t, ss))
    assert rc == _lib.TR_ERR_ARG and "sigma_s" in msg


def test_setup_rejects_bad_octant_order():
    from dataclasses import replace
    from paper_2010_04559_amd import _lib
    from paper_2010_04559_amd.transport import problem_struct
    L = _lib.load()
    p, keep = problem_struct(_small())
    p.octant_order[3] = p.octant_order[4]  # not a permutation
    h = ctypes.c_void_p()
    assert L.tr_setup(ctypes.byref(p), ctypes.byref(h)) == _lib.TR_ERR_ARG
    assert b"octant_order" in L.tr_last_error()
    with pytest.raises(ValueError):
        problem_struct(replace(_small(), octant_order=(0, 1, 2, 3, 4, 5, 6, 6)))


def test_setup_rejects_unknown_angular_basis():
    from paper_2010_04559_amd import _lib
    from paper_2010_04559_amd.transport import problem_struct
    L = _lib.load()
    p, keep = problem_struct(_small())
    p.angular_basis = 2
    h = ctypes.c_void_p()
    assert L.tr_setup(ctypes.byref(p), ctypes.byref(h)) == _lib.TR_ERR_ARG
    assert b"angular_basis" in L.tr_last_error() and not h.value


@pytest.mark.parametrize("orders", [[4, 97], [-1, 4]])
def test_setup_rejects_mg_order_out_of_range(orders):
    from dataclasses import replace
    from paper_2010_04559_amd import _lib
    rc, msg = _setup_rc(replace(_small(), mg_orders=orders))
    assert rc == _lib.TR_ERR_ARG and "mg_order" in msg


def test_setup_rejects_level_count_mismatch():
    from dataclasses import replace
    from paper_2010_04559_amd import _lib
    rc, msg = _setup_rc(replace(_small(), mg_orders=[4, 4, 4]))
    assert rc == _lib.TR_ERR_ARG and "n_levels" in msg and "2 levels" in msg


def test_setup_rejects_bad_smoothing_counts():
    from dataclasses import replace
    from paper_2010_04559_amd import _lib
    for kw in ({"nu_pre": 0}, {"nu_post": -1}, {"nu_coarse": 0}, {"nu_post_coarse": -1}):
        rc, msg = _setup_rc(replace(_small(), **kw))
        assert rc == _lib.TR_ERR_ARG and "nu_" in msg


def test_setup_rejects_bad_order_and_moments():
    from dataclasses import replace
    from paper_2010_04559_amd import _lib
    rc, msg = _setup_rc(replace(_small(), order=200, mg_orders=[4, 4]))
    assert rc == _lib.TR_ERR_ARG and "order" in msg
    rc, msg = _setup_rc(replace(_small(), hg_g=float("nan")))
    assert rc == _lib.TR_ERR_ARG and "moments" in msg


def test_workspace_bytes_without_a_device():
    """tr_workspace_bytes runs the host part of the setup only: sizes grow
    with the solve options as the allocations they count."""
    from paper_2010_04559_amd import inputs
    from paper_2010_04559_amd.transport import workspace_bytes
    prob = inputs.small_problem(dim=3, n=4, level=2, order=4)
    A, S = 3 * 128, 4 ** 3 * 8
    setup = workspace_bytes(prob)
    # at least: per level f, u, s (FP64), and the two finest work vectors
    assert setup >= 8 * S * (3 * (24 + 96 + 384) + 2 * A)
    f64 = workspace_bytes(prob, mode="f64", restart=10)
    rec = workspace_bytes(prob, mode="f64", restart=10, z_store="recompute")
    mixed = workspace_bytes(prob, mode="mixed", restart=10)
    # basis of 11 vectors + work vector; the kept FP64 Z adds 10 vectors,
    # the FP32 one 10 half-size vectors (the FP32 level buffers share the
    # FP64 level blocks)
    assert rec - setup >= 12 * 8 * A * S
    assert f64 - rec >= 10 * 8 * A * S
    assert 10 * 4 * A * S <= mixed - rec < 10 * 8 * A * S
    # the 48^3 precision problem with the FP32 preconditioner fits one
    # 288 GB device with room for the caller's right-hand side and solution
    big = workspace_bytes(inputs.config3(), mode="mixed")
    assert 1.5e11 < big < 288e9 - 2 * 8 * 1536 * 48 ** 3 * 8 - 10e9


def test_workspace_bytes_rejects_bad_options():
    from paper_2010_04559_amd import _lib, inputs
    from paper_2010_04559_amd.transport import problem_struct, solve_opts
    L = _lib.load()
    p, keep = problem_struct(inputs.small_problem())
    o = solve_opts(inputs.small_problem())
    o.z_store = 7
    out = ctypes.c_size_t()
    assert L.tr_workspace_bytes(ctypes.byref(p), ctypes.byref(o), ctypes.byref(out)) == _lib.TR_ERR_ARG
