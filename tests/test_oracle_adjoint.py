"""Pins of the oracle's adjoint solve and detector-response gradient."""
import numpy as np

from oracle import adjoint, krylov
from paper_2010_04559_amd import inputs
from oracle_problem import OracleProblem


def _prob(seed=0):
    p = inputs.small_problem(dim=2, n=3, level=1, g=0.85, order=6, c=0.9, seed=seed)
    p.n = (2, 2, 1)
    p.sigma_t, p.sigma_s, p.q_cell = p.sigma_t[:4], p.sigma_s[:4], p.q_cell[:4]
    p.detector = ((1, 0, 0), (1, 1, 0))
    return p


def test_reciprocity():
    op = OracleProblem(_prob())
    b, w = op.rhs(), op.detector()
    fwd = krylov.gmres(op.outer.apply_A, op.mg.vcycle, b, 1e-13, 10)
    adj = adjoint.solve_adjoint(op.outer, op.mg, w, 1e-13)
    assert fwd.converged and adj.converged
    assert abs(w @ fwd.x - adj.x @ b) < 1e-11 * abs(w @ fwd.x)


def test_gradient_matches_exact_derivative():
    """A is affine in each sigma, so A(sigma + e_j) - A(sigma) is dA/dsigma_j
    exactly; dR/dsigma_j = -lambda^T (dA/dsigma_j) phi with dense solves."""
    prob = _prob(1)
    op = OracleProblem(prob, with_mg=False)
    b, w = op.rhs(), op.detector()
    A = op.outer.dense(op.outer.apply_A)
    phi = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, w)
    gt, gs = adjoint.gradients(op.outer, lam, phi)
    for j in (0, 3):
        for which in ("t", "s"):
            st, ss = prob.sigma_t.copy(), prob.sigma_s.copy()
            (st if which == "t" else ss)[j] += 1.0
            op2 = OracleProblem(prob.with_sigma(st, ss), with_mg=False)
            dA = op2.outer.dense(op2.outer.apply_A) - A
            ref = -lam @ dA @ phi
            got = gt[j] if which == "t" else gs[j]
            assert abs(got - ref) < 1e-10 * max(1.0, abs(ref))


def test_gradient_matches_central_differences():
    prob = _prob(2)
    op = OracleProblem(prob)
    b, w = op.rhs(), op.detector()
    R, gt, gs, fwd, adj = adjoint.response_and_gradient(op.outer, op.mg, b, w, 1e-13)

    def resp(st, ss):
        o = OracleProblem(prob.with_sigma(st, ss), with_mg=False)
        return w @ np.linalg.solve(o.outer.dense(o.outer.apply_A), b)

    for j in (1, 2):
        h = 1e-6 * prob.sigma_t[j]
        st = prob.sigma_t.copy()
        st[j] += h
        rp = resp(st, prob.sigma_s)
        st[j] -= 2 * h
        rm = resp(st, prob.sigma_s)
        assert abs((rp - rm) / (2 * h) - gt[j]) < 1e-6 * np.abs(gt).max()
        h = 1e-6 * prob.sigma_s[j]
        ss = prob.sigma_s.copy()
        ss[j] += h
        rp = resp(prob.sigma_t, ss)
        ss[j] -= 2 * h
        rm = resp(prob.sigma_t, ss)
        assert abs((rp - rm) / (2 * h) - gs[j]) < 1e-6 * np.abs(gs).max()
