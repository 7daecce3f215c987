"""GPU checks at the full problem sizes, in the launch configuration the
benchmark times.

The 2-D configuration (16x16 cells, 32 patches, L = 8) is small enough for
the oracle to solve completely: iteration counts and solutions are compared
element by element.  At the 3-D sizes the oracle checks sampled (cell,
patch) blocks one by one: the block equation of every sweep output, the
scatter source of sampled cells, the operator rows of sampled blocks; the
solves are checked by their explicit residual through the (sample-checked)
operator, and gradients by central differences.
"""
import math

import numpy as np
import pytest

from oracle import angular as ang, spatial as sp, transport as otr, krylov
from paper_2010_04559_amd import inputs
from gpu_util import to_dev, to_np, rel, torch_mod
from oracle_problem import OracleProblem

pytestmark = pytest.mark.gpu


def _transport(prob):
    from paper_2010_04559_amd.transport import Transport
    return Transport(prob)


def _block(x, P, C, ns, q, j):
    return x.reshape(P, 3, C, ns)[q, :, j, :].reshape(-1)


def test_cfg1_full_solve_matches_oracle():
    prob = inputs.config1()
    print("case", prob.name, flush=True)
    tr = _transport(prob)
    op = OracleProblem(prob)
    b_np = op.rhs()
    assert rel(to_np(tr.rhs()), b_np) < 1e-13
    ref = krylov.gmres(op.outer.apply_A, op.mg.vcycle, b_np, 1e-8, prob.restart)
    x, st = tr.solve(to_dev(b_np))
    assert ref.converged and st["converged"] == 1
    assert st["iters"] == ref.iters
    assert rel(to_np(x), ref.x) < 1e-10
    xm, stm = tr.solve(to_dev(b_np), mode="mixed")
    assert stm["converged"] == 1
    phi = op.outer.scalar_flux_cell_avg(to_np(xm))
    assert rel(phi, op.outer.scalar_flux_cell_avg(ref.x)) < 1e-7


@pytest.fixture(scope="module")
def cfg2():
    prob = inputs.config2()
    print("case", prob.name, flush=True)
    tr = _transport(prob)
    grid = sp.Grid(prob.dim, prob.n, prob.length)
    patches = ang.AngularMesh.uniform(prob.angular.base_level).leaves()
    lv = otr.Level(grid, patches, prob.sigma_t, prob.sigma_s, prob.moments())
    rng = np.random.default_rng(21)
    samples = [(int(rng.integers(lv.P)), int(rng.integers(grid.C))) for _ in range(150)]
    # include boundary and corner cells
    samples += [(q, j) for q in (0, 37, 127) for j in (0, grid.C - 1, grid.C // 2)]
    return prob, tr, lv, samples


def _block_residual_L(lv, x, g, q, j):
    """(L x - g) restricted to block (j, q), from the oracle's block matrices."""
    G = lv.grid
    xb = lv.blocks(x)
    r = lv.K_stream[q] @ xb[q][j] + lv.sigma_t[j] * (lv.K_mass[q] @ xb[q][j])
    for xi, side, Cm in lv.couple[q]:
        nb = lv.nbr[(xi, side)][j]
        if nb >= 0:
            r = r + Cm @ xb[q][nb]
    return r - lv.blocks(g)[q][j]


def test_cfg2_sweep_blocks(cfg2):
    prob, tr, lv, samples = cfg2
    g = np.random.default_rng(22).standard_normal(lv.A * lv.grid.S)
    phi = to_np(tr.sweep(tr.nlev - 1, to_dev(g)))
    gb = lv.blocks(g)
    worst = 0.0
    for q, j in samples:
        r = _block_residual_L(lv, phi, g, q, j)
        worst = max(worst, np.abs(r).max() / np.abs(gb[q][j]).max())
    assert worst < 1e-11


def test_cfg2_sweep_fp32_blocks(cfg2):
    prob, tr, lv, samples = cfg2
    torch = torch_mod()
    g = np.random.default_rng(23).standard_normal(lv.A * lv.grid.S).astype(np.float32)
    phi = to_np(tr.sweep(tr.nlev - 1, to_dev(g, torch.float32)))
    gb = lv.blocks(g.astype(np.float64))
    worst = 0.0
    for q, j in samples:
        r = _block_residual_L(lv, phi, g.astype(np.float64), q, j)
        worst = max(worst, np.abs(r).max() / np.abs(gb[q][j]).max())
    assert worst < 1e-4


def test_cfg2_scatter_and_apply_blocks(cfg2):
    prob, tr, lv, samples = cfg2
    G = lv.grid
    x = np.random.default_rng(24).standard_normal(lv.A * G.S)
    s = to_np(tr.scatter(tr.nlev - 1, to_dev(x), outer=True)).reshape(lv.A, G.C, G.ns)
    y = to_np(tr.apply(to_dev(x)))
    xr = x.reshape(lv.A, G.C, G.ns)
    cells = sorted({j for _, j in samples})
    for j in cells:
        ref = lv.sigma_s[j] * (lv.Stilde @ xr[:, j, :]) @ G.N.T
        assert rel(s[:, j, :], ref) < 1e-12
    zero = np.zeros_like(x)
    for q, j in samples:
        # A = L - S on block (j, q)
        r = _block_residual_L(lv, x, zero, q, j)
        sq = (lv.sigma_s[j] * (lv.Stilde[3 * q:3 * q + 3] @ xr[:, j, :]) @ G.N.T).reshape(-1)
        ref = r - sq
        assert rel(_block(y, lv.P, G.C, G.ns, q, j), ref) < 1e-11


def test_cfg2_solves_converge(cfg2):
    prob, tr, lv, samples = cfg2
    torch = torch_mod()
    b = tr.rhs()
    x, st = tr.solve(b)
    res = float(torch.linalg.norm(b - tr.apply(x)) / torch.linalg.norm(b))
    assert st["converged"] == 1 and res < 1e-8
    xm, stm = tr.solve(b, mode="mixed")
    resm = float(torch.linalg.norm(b - tr.apply(xm)) / torch.linalg.norm(b))
    assert stm["converged"] == 1 and resm < 1e-8
    assert float(torch.linalg.norm(xm - x) / torch.linalg.norm(x)) < 1e-7
    # the source is symmetric about the cube centre but sigma_t is not:
    # check positivity of the cell-average scalar flux instead
    C, ns = lv.grid.C, lv.grid.ns
    ipsi = torch.as_tensor(lv.basis_integral(), device="cuda")
    phi0 = (ipsi[:, None] * x.reshape(lv.A, C * ns)).sum(0)
    assert float(phi0.min()) > -1e-6 * float(phi0.max())


def test_cfg2_coarse_gs_brick_form_matches_cell_form(cfg2):
    """The ten-sweep coarse Gauss-Seidel solve at 32^3 in the launch
    configuration the benchmark times (2 x 2 x 2 bricks on three waves
    each) against the per-cell dataflow form, forward and adjoint.  The two
    kernels differ in schedule, waits, in-brick exchanges and the mode
    solve (inverse row against LU); both match the oracle at small sizes."""
    import os
    prob, tr, lv, samples = cfg2
    torch = torch_mod()
    os.environ["TR_COARSE_GS"] = "cell"
    try:
        tc = _transport(prob)
    finally:
        os.environ.pop("TR_COARSE_GS", None)
    try:
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        f = torch.randn(tc.n(0), dtype=torch.float64, device="cuda", generator=g)
        for adj in (False, True):
            print("coarse GS 32^3, adjoint" if adj else "coarse GS 32^3, forward", flush=True)
            a = tr.coarse_gs(f, prob.nu_coarse, adjoint=adj)
            c = tc.coarse_gs(f, prob.nu_coarse, adjoint=adj)
            assert float(torch.linalg.norm(a - c) / torch.linalg.norm(c)) < 1e-12, adj
    finally:
        tc.close()


def test_cfg4_gradient_fd_full_size():
    prob = inputs.config4()
    print("case", prob.name, flush=True)
    tr = _transport(prob)
    torch = torch_mod()
    b, w = tr.rhs(), tr.detector()
    x, st = tr.solve(b, tol=1e-13, mode="mixed")
    assert st["converged"] == 1
    gt, gs, lam, sta = tr.adjoint_grad(w, x, tol=1e-13, mode="mixed")
    assert sta["converged"] == 1
    R = float(torch.dot(w, x))
    assert abs(R - float(torch.dot(lam, b))) < 1e-10 * abs(R)
    gt, gs = to_np(gt), to_np(gs)
    st0, ss0 = prob.sigma_t.copy(), prob.sigma_s.copy()
    for j in prob.fd_cells[:2]:
        for which in ("t", "s"):
            base = (st0 if which == "t" else ss0)[j]
            h = 1e-6 * base
            vals = []
            for sgn in (1, -1):
                st_, ss_ = st0.copy(), ss0.copy()
                (st_ if which == "t" else ss_)[j] = base + sgn * h
                tr.set_sigma(st_, ss_)
                xs, _ = tr.solve(b, tol=1e-13, mode="mixed")
                vals.append(float(torch.dot(w, xs)))
            fd = (vals[0] - vals[1]) / (2 * h)
            ref = gt if which == "t" else gs
            assert abs(fd - ref[j]) < 1e-5 * np.abs(ref).max(), (which, j, fd, ref[j])
    tr.set_sigma(st0, ss0)


def test_cfg5_cone_mesh_solve_and_scatter_row():
    prob = inputs.config5()
    print("case", prob.name, flush=True)
    tr = _transport(prob)
    torch = torch_mod()
    assert tr.patches == [8, 32, 128, 152, 200, 368]
    b = tr.rhs()
    x, st = tr.solve(b, mode="mixed")
    res = float(torch.linalg.norm(b - tr.apply(x)) / torch.linalg.norm(b))
    assert st["converged"] == 1 and res < 1e-8
    G = sp.Grid(prob.dim, prob.n, prob.length)
    mesh = ang.AngularMesh.cone(prob.angular.cone_axis, prob.angular.cone_half_angle_deg,
                                prob.angular.base_level, prob.angular.extra_levels)
    leaves = mesh.leaves()
    A = 3 * len(leaves)
    # order-64 problem operator: an isotropic flux scatters isotropically, so
    # S 1 = sigma_s (int psi) (N 1): every harmonic of degree 1..64 must
    # integrate to zero over the sphere in the library's X integrals
    ipsi = np.concatenate([ang.lin_basis(p, om).T @ w for p in leaves for om, w in [ang.quad_accurate(p)]])
    s1 = to_np(tr.scatter(tr.nlev - 1, to_dev(np.ones(A * G.S)), outer=True)).reshape(A, G.C, G.ns)
    ref1 = prob.sigma_s[None, :, None] * ipsi[:, None, None] * (G.N.sum(axis=1))[None, None, :]
    assert rel(s1, ref1) < 1e-11
    # one row block of the finest multigrid level's scatter matrix (order
    # 16) through the addition theorem, for a patch inside the cone
    qs = 200
    rows = ang.scatter_rows_addition(leaves, prob.moments(prob.mg_orders[-1]), qs)
    xr = np.random.default_rng(25).standard_normal(A * G.S)
    s = to_np(tr.scatter(tr.nlev - 1, to_dev(xr), outer=False)).reshape(A, G.C, G.ns)
    X = xr.reshape(A, G.C, G.ns)
    for j in (0, 777, G.C - 1):
        ref = prob.sigma_s[j] * (rows @ X[:, j, :]) @ G.N.T
        assert rel(s[3 * qs:3 * qs + 3, j, :], ref) < 1e-10
