"""GPU checks of the solver's storage modes and of the boundary's helper
calls, against the oracle:

* the FP32 preconditioner runs flexible GMRES with its preconditioned
  vectors kept in FP32 (deterministically, whatever the free memory), and
  gives the oracle's solution to 1e-7; the non-flexible comparison form
  (z_store = "recompute") and the FP64 forms with and without kept vectors
  give the oracle's iterations and solution;
* the preconditioner sees unit-norm inputs: right-hand sides scaled by
  1e-30 and 1e+30 take the unscaled iteration counts and solutions;
* the detector response, its gradients with respect to b and w through
  autograd, the device memory the handle reports against tr_workspace_bytes,
  the checks of tr_set_sigma;
* the beam right-hand side (Section 5.5) against the oracle's, on a small
  grid and on the 32^3 beam problem's face box.
"""
import numpy as np
import pytest

from oracle import krylov, adjoint
from paper_2010_04559_amd import inputs
from gpu_util import Pair, small, to_dev, to_np, rel, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair3():
    prob = small(dim=3, n=4, level=2, order=8, g=0.9, c=0.97, seed=31)
    print("case", prob.name, flush=True)
    return Pair(prob)


@pytest.fixture(scope="module")
def ref3(pair3):
    b = pair3.op.rhs()
    return b, krylov.gmres(pair3.op.outer.apply_A, pair3.op.mg.vcycle, b, 1e-10, pair3.prob.restart)


@pytest.mark.parametrize("z_store", ["auto", "keep", "recompute"])
def test_fp64_storage_forms_match_oracle(pair3, ref3, z_store):
    b, ref = ref3
    x, st = pair3.tr.solve(to_dev(b), tol=1e-10, z_store=z_store)
    assert st["converged"] == 1 and st["iters"] == ref.iters
    assert st["flexible"] == (0 if z_store == "recompute" else 64)
    assert rel(to_np(x), ref.x) < 1e-10


@pytest.mark.parametrize("mode", ["mixed", "mixed_bf16"])
def test_fp32_preconditioner_is_flexible(pair3, ref3, mode):
    b, ref = ref3
    x, st = pair3.tr.solve(to_dev(b), tol=1e-10, mode=mode)
    assert st["converged"] == 1 and st["flexible"] == 32
    assert st["iters"] <= ref.iters + 1
    assert rel(to_np(x), ref.x) < 1e-7
    # the comparison form without kept vectors still converges
    xr, sr = pair3.tr.solve(to_dev(b), tol=1e-10, mode=mode, z_store="recompute")
    assert sr["converged"] == 1 and sr["flexible"] == 0
    assert rel(to_np(xr), ref.x) < 1e-7


@pytest.mark.parametrize("scale", [1e-30, 1e30])
@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_scaled_right_hand_side(pair3, ref3, scale, mode):
    b, ref = ref3
    x0, s0 = pair3.tr.solve(to_dev(b), tol=1e-10, mode=mode)
    xs, ss = pair3.tr.solve(to_dev(b * scale), tol=1e-10, mode=mode)
    assert ss["converged"] == 1 and ss["iters"] == s0["iters"]
    assert rel(to_np(xs) / scale, to_np(x0)) < 1e-9
    assert rel(to_np(xs) / scale, ref.x) < 1e-7


def test_response_and_autograd_inputs(pair3, ref3):
    """R = w . phi through the library; dR/db = lambda and dR/dw = phi."""
    torch = torch_mod()
    from paper_2010_04559_amd.autograd import DetectorResponse
    b, ref = ref3
    lo, hi = (2, 1, 1), (3, 2, 3)
    w_np = pair3.op.outer.detector_weights(lo, hi)
    x = pair3.tr.solve(to_dev(b), tol=1e-12)[0]
    assert abs(pair3.tr.response(to_dev(w_np), x) - w_np @ ref.x) < 1e-9 * abs(w_np @ ref.x)
    st = torch.tensor(pair3.prob.sigma_t, dtype=torch.float64, device="cuda", requires_grad=True)
    ss = torch.tensor(pair3.prob.sigma_s, dtype=torch.float64, device="cuda", requires_grad=True)
    bt = to_dev(b).requires_grad_(True)
    wt = to_dev(w_np).requires_grad_(True)
    R = DetectorResponse.apply(pair3.tr, st, ss, bt, wt, "f64", 1e-12)
    R.backward()
    lam = adjoint.solve_adjoint(pair3.op.outer, pair3.op.mg, w_np, 1e-12, pair3.prob.restart).x
    assert rel(to_np(bt.grad), lam) < 1e-9
    assert rel(to_np(wt.grad), ref.x) < 1e-8
    _, gt, gs, _, _ = adjoint.response_and_gradient(pair3.op.outer, pair3.op.mg, b, w_np, 1e-12)
    assert rel(to_np(st.grad), gt) < 1e-8 and rel(to_np(ss.grad), gs) < 1e-8


def test_set_sigma_checks_values(pair3, ref3):
    from paper_2010_04559_amd import _lib
    b, ref = ref3
    prob = pair3.prob
    bad = prob.sigma_t.copy()
    bad[7] = float("nan")
    with pytest.raises(_lib.TrError) as e:
        pair3.tr.set_sigma(bad, prob.sigma_s)
    assert e.value.code == _lib.TR_ERR_ARG
    neg = prob.sigma_s.copy()
    neg[2] = -1.0
    with pytest.raises(_lib.TrError):
        pair3.tr.set_sigma(prob.sigma_t, neg)
    # the handle kept its cross sections
    x, st = pair3.tr.solve(to_dev(b), tol=1e-10)
    assert st["iters"] == ref.iters and rel(to_np(x), ref.x) < 1e-10


@pytest.mark.parametrize("mode", [None, "f64", "mixed", "mixed_bf16"])
def test_workspace_bytes_match_the_handle(mode):
    """tr_workspace_bytes (host only) counts what a fresh handle holds after
    setup and after one forward solve in the given mode."""
    from paper_2010_04559_amd.transport import Transport, workspace_bytes
    prob = small(dim=3, n=4, level=2, order=6, seed=33)
    print("case", prob.name, mode, flush=True)
    tr = Transport(prob)
    assert tr.device_bytes() == workspace_bytes(prob)
    if mode is not None:
        b = tr.rhs()
        tr.solve(b, mode=mode, z_store="keep" if mode == "f64" else "auto")
        assert tr.device_bytes() == workspace_bytes(prob, mode=mode)
    tr.close()


@pytest.mark.parametrize("which", ["small", "cfg4"])
def test_beam_rhs_matches_oracle(which):
    if which == "small":
        prob = small(dim=3, n=(5, 6, 6), level=2, order=4, seed=35, inflow=False)
        from dataclasses import replace
        prob = replace(prob, inflow=inputs.Inflow("beam", 0, 0, (0, 1, 2), (0, 4, 4), 1.3, (1.0, 0.0, 0.0)))
    else:
        prob = inputs.config4()
    print("case beam", prob.name, flush=True)
    pr = Pair(prob, with_mg=False)
    got = to_np(pr.tr.rhs())
    want = pr.op.rhs()
    assert rel(got, want) < 1e-13
    # total source = current x face-box area (Section 5.5, unit current per area)
    f = prob.inflow
    area = (f.hi[1] - f.lo[1] + 1) * (f.hi[2] - f.lo[2] + 1) / (prob.n[1] * prob.n[2])
    assert abs(got.sum() - f.value * area - (want.sum() - f.value * area)) < 1e-12
    assert abs(want.sum() - f.value * area - pr.op.outer.rhs_volume(prob.q_cell).sum()) < 1e-12 * abs(want.sum())
