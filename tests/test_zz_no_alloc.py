"""The allocation-free coarse Gauss-Seidel solve (tr_coarse_gs_noalloc)
against tr_coarse_gs on the same handle: the same kernels with the update
counters and the error word in the library's per-device scratch instead of
the handle's buffers.  Two calls in a row, the second on a smaller problem
(fewer counters), in the brick form (even 3-D grids) and the cell form (an
odd grid), forward and adjoint; and the errors it reports instead of
allocating."""
import ctypes

import numpy as np
import pytest

from gpu_util import small, to_dev, to_np, rel, torch_mod

pytestmark = pytest.mark.gpu


def _noalloc(tr, f, nu, adjoint=False):
    from paper_2010_04559_amd import _lib
    fn = tr.lib.tr_coarse_gs_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    out = torch_mod().empty_like(f)
    stream = ctypes.c_void_p(torch_mod().cuda.current_stream().cuda_stream)
    rc = fn(tr.h, nu, 1 if adjoint else 0, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), stream)
    return rc, out


def _handle(n, seed):
    from paper_2010_04559_amd.transport import Transport
    prob = small(dim=3, n=n, level=0, order=3, seed=seed)
    print("case", prob.name, flush=True)
    return Transport(prob)


@pytest.mark.parametrize("adjoint", [False, True])
def test_noalloc_matches_coarse_gs_two_calls(adjoint):
    from paper_2010_04559_amd import _lib
    big = _handle((6, 4, 8), 41)     # 24 bricks
    little = _handle((4, 4, 2), 42)  # 4 bricks
    odd = _handle(3, 43)             # 27 cells: the per-cell form
    for tr, seed in ((big, 1), (little, 2), (odd, 3)):
        nu = tr.prob.nu_coarse
        f = to_dev(np.random.default_rng(seed).standard_normal(24 * tr.S))
        want = to_np(tr.coarse_gs(f, nu, adjoint=adjoint))
        rc, got = _noalloc(tr, f, nu, adjoint)
        assert rc == _lib.TR_OK, tr.lib.tr_last_error()
        assert rel(to_np(got), want) < 1e-13
    # the scratch keeps the last call's counters: a repeat on the big
    # problem after the small one still agrees
    f = to_dev(np.random.default_rng(4).standard_normal(24 * big.S))
    rc, got = _noalloc(big, f, big.prob.nu_coarse, adjoint)
    assert rc == _lib.TR_OK
    assert rel(to_np(got), to_np(big.coarse_gs(f, big.prob.nu_coarse, adjoint=adjoint))) < 1e-13
    for tr in (big, little, odd):
        tr.close()


def test_noalloc_reports_instead_of_allocating():
    from paper_2010_04559_amd import _lib
    tr = _handle((4, 4, 4), 44)
    f = to_dev(np.random.default_rng(5).standard_normal(24 * tr.S))
    # a sweep count whose schedule is not prepared
    rc, _ = _noalloc(tr, f, 3)
    assert rc == _lib.TR_ERR_ARG and b"schedule" in tr.lib.tr_last_error()
    # after one tr_coarse_gs call with that count it is
    want = to_np(tr.coarse_gs(f, 3))
    rc, got = _noalloc(tr, f, 3)
    assert rc == _lib.TR_OK and rel(to_np(got), want) < 1e-13
    # more than 15 sweeps run the barrier form only
    tr.coarse_gs(f, 16)
    rc, _ = _noalloc(tr, f, 16)
    assert rc == _lib.TR_ERR_UNSUPPORTED
    tr.close()
