"""GPU parity of the Const angular basis (Section 2.2) against the oracle's
one-dof-per-patch Const discretisation.

The library carries a Const function as three coincident ordinates per
patch holding equal values (include/tr.h, TR_BASIS_CONST): a Const
solution c_q is the library vector with all three coefficients of patch q
equal to c_q, a Const weak-form vector b_q the one with b_q / 3 in each.
Every operator is compared through that correspondence, element by
element (FP64: relative 1e-12; FP32: 2e-5), and every library result is
checked to stay in that form.  Solves take the oracle's iteration counts
and agree to 1e-10 (FP64 preconditioner) and 1e-7 (FP32)."""
import numpy as np
import pytest

from oracle import krylov, adjoint as oadj
from paper_2010_04559_amd import inputs
from gpu_util import Pair, small, to_dev, to_np, rel, torch_mod

pytestmark = pytest.mark.gpu

CASES = [
    dict(dim=3, n=4, level=1, order=6, seed=51),               # even grid: pair sweep
    dict(dim=2, n=3, level=2, order=8, g=0.9, seed=52),
    dict(dim=3, n=3, level=1, order=4, seed=53, beam=True),    # odd grid: cell sweep, beam source
]


def _problem(kw):
    kw = dict(kw)
    beam = kw.pop("beam", False)
    level = kw.pop("level")
    prob = small(angular=inputs.AngularSpec(level, basis="const"), level=level, **kw)
    if beam:
        prob.inflow = inputs.Inflow("beam", 0, 0, (0, 0, 0), (0, 2, 2), 1.0, (1.0, 0.0, 0.0))
    return prob


@pytest.fixture(scope="module", params=range(len(CASES)))
def pair(request):
    prob = _problem(CASES[request.param])
    print("case", prob.name, flush=True)
    return Pair(prob)


def sol(x, S):
    """Const solution (P rows) -> library layout (three equal rows per patch)."""
    return np.repeat(np.asarray(x).reshape(-1, S), 3, axis=0).reshape(-1)


def weak(b, S):
    """Const weak-form vector -> library layout (a third in each row)."""
    return sol(b, S) / 3.0


def back(x, S, weak_form=False):
    """Library vector -> Const (P rows), after checking the three rows of
    every patch agree."""
    x = np.asarray(x).reshape(-1, 3, S)
    spread = np.abs(x - x[:, :1, :]).max()
    assert spread <= 1e-12 * max(np.abs(x).max(), 1e-300), spread
    return (x[:, 0, :] * (3.0 if weak_form else 1.0)).reshape(-1)


def _rand(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def test_const_rhs_and_detector(pair):
    S = pair.tr.S
    assert rel(to_np(pair.tr.rhs()), weak(pair.op.rhs(), S)) < 1e-13
    lo, hi = (0, 1, 0), (1, 2, 1)
    assert rel(to_np(pair.tr.detector(lo, hi)), weak(pair.op.outer.detector_weights(lo, hi), S)) < 1e-13


def test_const_sweeps_and_scatter(pair):
    torch = torch_mod()
    S = pair.tr.S
    for l in range(pair.tr.nlev):
        lv = pair.level(l)
        g = _rand(lv.A * S, 10 + l)
        ref = lv.sweep(g)
        got = to_np(pair.tr.sweep(l, to_dev(weak(g, S))))
        assert rel(back(got, S), ref) < 1e-12, l
        got = to_np(pair.tr.sweep(l, to_dev(weak(g, S)), adjoint=True))
        assert rel(back(got, S), lv.sweep_T(g)) < 1e-12, l
        x = _rand(lv.A * S, 20 + l)
        got = to_np(pair.tr.scatter(l, to_dev(sol(x, S))))
        assert rel(back(got, S, weak_form=True), lv.apply_S(x)) < 1e-12, l
    L = pair.tr.nlev - 1
    lv = pair.level(L)
    g = _rand(lv.A * S, 30)
    got32 = to_np(pair.tr.sweep(L, to_dev(weak(g, S), torch.float32)))
    assert rel(got32.reshape(-1, 3, S)[:, 0, :].reshape(-1), lv.sweep(g)) < 2e-5
    out = pair.level(0, outer=True)
    x = _rand(out.A * S, 31)
    got = to_np(pair.tr.scatter(L, to_dev(sol(x, S)), outer=True))
    assert rel(back(got, S, weak_form=True), out.apply_S(x)) < 1e-12
    got = to_np(pair.tr.apply(to_dev(sol(x, S))))
    assert rel(back(got, S, weak_form=True), out.apply_A(x)) < 1e-12


def test_const_transfers_and_coarse_solve(pair):
    mg = pair.op.mg
    S = mg.grid.S
    for l in range(1, pair.tr.nlev):
        xc = _rand(mg.levels[l - 1].A * S, 40 + l)
        got = to_np(pair.tr.prolong(l, to_dev(sol(xc, S))))
        assert rel(back(got, S), mg.prolong(l, xc)) < 1e-14
        rf = _rand(mg.levels[l].A * S, 50 + l)
        got = to_np(pair.tr.restrict(l, to_dev(weak(rf, S))))
        assert rel(back(got, S, weak_form=True), mg.restrict(l, rf)) < 1e-14
    f = _rand(mg.levels[0].A * S, 60)
    for adj in (False, True):
        got = to_np(pair.tr.coarse_gs(to_dev(weak(f, S)), 3, adjoint=adj))
        assert rel(back(got, S), mg.coarse_gs(f, 3, adjoint=adj)) < 1e-11


def test_const_vcycles(pair):
    S = pair.tr.S
    lv = pair.level(0, outer=True)
    r = _rand(lv.A * S, 70)
    rd = to_dev(weak(r, S))
    assert rel(back(to_np(pair.tr.vcycle(rd)), S), pair.op.mg.vcycle(r)) < 1e-11
    assert rel(back(to_np(pair.tr.vcycle(rd, adjoint=True)), S), pair.op.mg.vcycle(r, adjoint=True)) < 1e-11
    assert rel(back(to_np(pair.tr.vcycle(rd, mode="sg")), S), lv.sweep(r)) < 1e-12
    got = to_np(pair.tr.vcycle(rd, mode="mixed")).reshape(-1, 3, S)[:, 0, :].reshape(-1)
    assert rel(got, pair.op.mg.vcycle(r)) < 1e-4


def test_const_solves_match_oracle(pair):
    S = pair.tr.S
    b = pair.op.rhs()
    bd = to_dev(weak(b, S))
    A, M = pair.op.outer.apply_A, pair.op.mg.vcycle
    ref = krylov.gmres(A, M, b, 1e-10, pair.prob.restart)
    assert ref.converged
    x, st = pair.tr.solve(bd, tol=1e-10)
    assert st["converged"] == 1 and st["iters"] == ref.iters
    assert rel(back(to_np(x), S), ref.x) < 1e-10
    xm, sm = pair.tr.solve(bd, tol=1e-10, mode="mixed")
    assert sm["converged"] == 1
    assert rel(to_np(xm).reshape(-1, 3, S)[:, 0, :].reshape(-1), ref.x) < 1e-7
    refb = krylov.bicgstab(A, M, b, 1e-10)
    xb, sb = pair.tr.solve(bd, tol=1e-10, method="bicgstab")
    assert sb["converged"] == 1 and sb["iters"] == refb.iters
    assert rel(back(to_np(xb), S), refb.x) < 1e-10


def test_const_adjoint_gradient(pair):
    S = pair.tr.S
    lo, hi = (0, 0, 0), (2, 2, 2)
    out = pair.op.outer
    w = out.detector_weights(lo, hi)
    b = pair.op.rhs()
    R, gt, gs, fwd, adj = oadj.response_and_gradient(out, pair.op.mg, b, w, tol=1e-12)
    x, _ = pair.tr.solve(to_dev(weak(b, S)), tol=1e-12)
    gt_d, gs_d, lam, _ = pair.tr.adjoint_grad(to_dev(weak(w, S)), x, tol=1e-12)
    assert rel(to_np(gt_d), gt) < 1e-9
    assert rel(to_np(gs_d), gs) < 1e-9
    assert rel(back(to_np(lam), S), adj.x) < 1e-9
