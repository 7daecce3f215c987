"""GPU parity of the full solver (GMRES + angular multigrid), the mixed
precision preconditioner and the adjoint gradient against the oracle."""
import numpy as np
import pytest

from oracle import krylov, adjoint
from paper_2010_04559_amd import inputs
from gpu_util import Pair, small, to_dev, to_np, rel, torch_mod

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kw", [dict(dim=2, n=4, level=2, order=8, g=0.9, c=0.98, seed=5),
                                dict(dim=3, n=3, level=1, order=6, g=0.9, c=0.95, seed=6)])
def test_gmres_matches_oracle(kw):
    print("case", kw, flush=True)
    prob = small(**kw)
    pr = Pair(prob)
    b_np = pr.op.rhs()
    ref = krylov.gmres(pr.op.outer.apply_A, pr.op.mg.vcycle, b_np, 1e-8, prob.restart)
    x, st = pr.tr.solve(to_dev(b_np), tol=1e-8)
    assert st["converged"] == 1 and ref.converged
    assert st["iters"] == ref.iters
    assert rel(to_np(x), ref.x) < 1e-10


def test_mixed_precision_solution_matches_fp64_oracle():
    prob = small(dim=2, n=4, level=2, order=8, g=0.9, c=0.98, seed=7)
    pr = Pair(prob)
    b_np = pr.op.rhs()
    ref = krylov.gmres(pr.op.outer.apply_A, pr.op.mg.vcycle, b_np, 1e-12, prob.restart)
    x, st = pr.tr.solve(to_dev(b_np), tol=1e-8, mode="mixed")
    assert st["converged"] == 1 and st["rel_res"] < 1e-8
    phi_ref = pr.op.outer.scalar_flux_cell_avg(ref.x)
    phi = pr.op.outer.scalar_flux_cell_avg(to_np(x))
    assert rel(phi, phi_ref) < 1e-7


def test_split_bf16_preconditioner_solution_matches_fp64_oracle():
    """FP32 V-cycle with split-BF16 scatter products inside FP64 GMRES: the
    converged solution meets the FP64 oracle's to 1e-7, and the iteration
    count is that of the FP32 preconditioner (the condition under which the
    split products are used)."""
    prob = small(dim=3, n=4, level=2, order=10, g=0.9, c=0.98, seed=19)
    pr = Pair(prob)
    b_np = pr.op.rhs()
    ref = krylov.gmres(pr.op.outer.apply_A, pr.op.mg.vcycle, b_np, 1e-12, prob.restart)
    x32, st32 = pr.tr.solve(to_dev(b_np), tol=1e-8, mode="mixed")
    x, st = pr.tr.solve(to_dev(b_np), tol=1e-8, mode="mixed_bf16")
    print("iterations fp32", st32["iters"], "split-bf16", st["iters"], flush=True)
    assert st["converged"] == 1 and st["rel_res"] < 1e-8
    assert st["iters"] == st32["iters"]
    phi_ref = pr.op.outer.scalar_flux_cell_avg(ref.x)
    phi = pr.op.outer.scalar_flux_cell_avg(to_np(x))
    assert rel(phi, phi_ref) < 1e-7


def test_single_grid_preconditioner_matches_oracle():
    prob = small(dim=2, n=3, level=1, order=4, g=0.8, c=0.9, seed=8)
    pr = Pair(prob)
    b_np = pr.op.rhs()
    ref = krylov.gmres(pr.op.outer.apply_A, pr.op.outer.sweep, b_np, 1e-8, prob.restart)
    x, st = pr.tr.solve(to_dev(b_np), tol=1e-8, mode="sg")
    assert st["iters"] == ref.iters
    assert rel(to_np(x), ref.x) < 1e-10


def test_adjoint_gradient_matches_oracle():
    prob = small(dim=2, n=4, level=1, order=6, g=0.85, c=0.9, seed=9)
    prob.detector = ((2, 1, 0), (3, 2, 0))
    pr = Pair(prob)
    b_np, w_np = pr.op.rhs(), pr.op.detector()
    R, gt_ref, gs_ref, fwd, adj = adjoint.response_and_gradient(pr.op.outer, pr.op.mg, b_np, w_np, 1e-12)
    x, _ = pr.tr.solve(to_dev(b_np), tol=1e-12)
    gt, gs, lam, st = pr.tr.adjoint_grad(to_dev(w_np), x, tol=1e-12)
    assert st["converged"] == 1
    assert st["iters"] == adj.iters
    assert rel(to_np(lam), adj.x) < 1e-9
    assert rel(to_np(gt), gt_ref) < 1e-9
    assert rel(to_np(gs), gs_ref) < 1e-9


def test_gradient_matches_central_differences_on_gpu():
    prob = small(dim=2, n=4, level=1, order=6, g=0.85, c=0.9, seed=10)
    prob.detector = ((2, 1, 0), (3, 2, 0))
    pr = Pair(prob, with_mg=False)
    tr = pr.tr
    b, w = tr.rhs(), tr.detector()
    x, _ = tr.solve(b, tol=1e-13)
    gt, gs, _, _ = tr.adjoint_grad(w, x, tol=1e-13)
    gt, gs = to_np(gt), to_np(gs)
    torch = torch_mod()
    for j in (3, 9):
        for which in ("t", "s"):
            st0, ss0 = prob.sigma_t.copy(), prob.sigma_s.copy()
            base = (st0 if which == "t" else ss0)[j]
            h = 1e-6 * base
            vals = []
            for sgn in (1, -1):
                st, ss = st0.copy(), ss0.copy()
                (st if which == "t" else ss)[j] = base + sgn * h
                tr.set_sigma(st, ss)
                xs, _ = tr.solve(b, tol=1e-13)
                vals.append(float(torch.dot(w, xs)))
            tr.set_sigma(st0, ss0)
            fd = (vals[0] - vals[1]) / (2 * h)
            ref = gt if which == "t" else gs
            assert abs(fd - ref[j]) < 1e-5 * np.abs(ref).max(), (which, j, fd, ref[j])


def test_autograd_detector_response_matches_oracle():
    """torch.autograd through DetectorResponse: R and both gradients against
    the oracle's adjoint gradient on the same problem."""
    torch = torch_mod()
    from paper_2010_04559_amd.autograd import detector_response
    prob = small(dim=2, n=4, level=1, order=6, g=0.85, c=0.9, seed=11)
    prob.detector = ((2, 1, 0), (3, 2, 0))
    pr = Pair(prob)
    b_np, w_np = pr.op.rhs(), pr.op.detector()
    R_ref, gt_ref, gs_ref, _, _ = adjoint.response_and_gradient(pr.op.outer, pr.op.mg, b_np, w_np, 1e-12)
    st = torch.tensor(prob.sigma_t, dtype=torch.float64, device="cuda", requires_grad=True)
    ss = torch.tensor(prob.sigma_s, dtype=torch.float64, device="cuda", requires_grad=True)
    R = detector_response(pr.tr, st, ss, to_dev(b_np), to_dev(w_np), "f64", 1e-12)
    assert abs(float(R.detach()) - R_ref) < 1e-10 * abs(R_ref)
    (3.0 * R).backward()
    assert rel(to_np(st.grad), 3.0 * gt_ref) < 1e-9
    assert rel(to_np(ss.grad), 3.0 * gs_ref) < 1e-9
