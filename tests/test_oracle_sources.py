"""Pins of the oracle's source terms and of the whole discrete system.

* The Dirac beam of Section 5.5 (rhs_beam): the total weak-form source is
  the entering current times the face area (test functions sum to one in
  space and in angle); a direction strictly inside a patch is represented
  by that patch's Lin functions at the direction (barycentric weights,
  which reproduce every gnomonic-linear function); a direction on a vertex
  shared by four patches is split into equal quarters.
* The Fokker-Planck-equivalent moments of eq. scatter_moments (fp_moments):
  the scatter operator minus sigma_{s,0} acts on each spherical harmonic of
  degree n as alpha/2 times the Laplace-Beltrami operator, which the test
  evaluates by finite differences of the harmonics (not from the formula).
* Particle balance of a converged solve: the sum of all weak equations is
  outflow leakage + removal - scatter-in = volume source + beam current,
  every term formed here from the basic integrals (face integrals of the
  spatial basis, the angular rule, cross sections), not from the operator.
"""
import math

import numpy as np
import pytest

from oracle import angular as ang
from oracle import spatial as sp
from oracle import transport as tr
from oracle import krylov
from paper_2010_04559_amd import inputs
from oracle_problem import OracleProblem


def _level(dim, n, level, order=4, g=0.8, seed=0, c=0.9):
    grid = sp.Grid(dim, n)
    rng = np.random.default_rng(seed)
    st = rng.uniform(0.5, 3.0, grid.C)
    ss = c * st * rng.uniform(0.5, 1.0, grid.C)
    return tr.Level(grid, ang.AngularMesh.uniform(level).leaves(), st, ss, ang.hg_moments(g, order))


# ------------------------------------------------------------------ beam

@pytest.mark.parametrize("dim,n,lo,hi", [(3, (6, 8, 8), (0, 2, 3), (0, 5, 6)), (2, (5, 7), (0, 1, 0), (0, 4, 0)),
                                         (3, (8, 8, 8), (0, 2, 2), (0, 5, 5))])
def test_beam_total_source_is_current_times_area(dim, n, lo, hi):
    lv = _level(dim, n, 2)
    current = 1.7
    b = lv.rhs_beam((1.0, 0.0, 0.0), 0, 0, lo, hi, current)
    g = lv.grid
    area = 1.0
    for a in range(1, dim):
        area *= (hi[a] - lo[a] + 1) * g.h[a]
    assert abs(b.sum() - current * area) < 1e-14 * current * area
    # every entry sits on the inflow face x = 0 of a box cell
    bx = b.reshape(lv.A, g.C, g.ns)
    cells = np.unique(np.nonzero(np.abs(bx).sum(axis=(0, 2)))[0])
    assert (g.coords[cells, 0] == 0).all()
    for a in range(1, dim):
        assert ((g.coords[cells, a] >= lo[a]) & (g.coords[cells, a] <= hi[a])).all()
    # and on the nodes of that face only
    assert np.abs(bx[:, :, 1::2]).max() == 0.0


def test_beam_on_a_shared_vertex_splits_into_quarters():
    """+x is a vertex of one patch in each of the four octants with s_x > 0;
    the Lin function of that vertex is one there and the others vanish."""
    lv = _level(3, (4, 4, 4), 2)
    b = lv.rhs_beam((1.0, 0.0, 0.0), 0, 0, (0, 0, 0), (0, 3, 3), 1.0)
    per_dof = b.reshape(lv.A, -1).sum(axis=1)
    hit = np.nonzero(per_dof)[0]
    assert len(hit) == 4
    assert np.allclose(per_dof[hit], 0.25, rtol=0, atol=1e-15)
    octs = set()
    for a in hit:
        p = lv.patches[a // 3]
        assert np.allclose(p.verts[a % 3], [1.0, 0.0, 0.0], atol=1e-15)
        octs.add(p.octant)
    assert octs == {0, 2, 4, 6}


def test_beam_inside_a_patch_uses_barycentric_weights():
    """A direction strictly inside one patch: only that patch is hit, with
    weights that reproduce gnomonic-linear functions at the direction."""
    lv = _level(3, (3, 3, 3), 2)
    rng = np.random.default_rng(3)
    for trial in range(5):
        q = int(rng.integers(lv.P))
        p = lv.patches[q]
        s = ang.octant_signs(p.octant)
        if s[0] < 0:
            continue  # the beam must enter through x = 0
        lam = rng.dirichlet([2.0, 2.0, 2.0])
        flat = ang.gnomonic(p.verts, s)
        x = lam @ flat
        d = x / np.linalg.norm(x)
        b = lv.rhs_beam(d, 0, 0, (0, 0, 0), (0, 2, 2), 1.0)
        per_dof = b.reshape(lv.A, -1).sum(axis=1)
        assert set(np.nonzero(per_dof)[0]) <= {3 * q, 3 * q + 1, 3 * q + 2}
        wts = per_dof[3 * q:3 * q + 3] / per_dof.sum()
        # f(Omega) = c . gnomonic(Omega) + c0, linear on the face plane
        c, c0 = rng.standard_normal(3), rng.standard_normal()
        f_vertices = flat @ c + c0
        f_dir = ang.gnomonic(d, s)[0] @ c + c0
        assert abs(wts @ f_vertices - f_dir) < 1e-12 * (1 + abs(f_dir))


# ------------------------------------------------------ Fokker-Planck moments

def _laplace_beltrami_fd(order, pts, h=1e-3):
    """Delta_S of every real harmonic at unit vectors pts, as the Cartesian
    Laplacian of the degree-0 homogeneous extension F(x) = Y(x / |x|)
    (equal to Delta_S Y on the unit sphere), fourth-order central
    differences."""
    def F(x):
        return ang.real_harmonics(order, x / np.linalg.norm(x, axis=1)[:, None])
    lap = -3 * 2.5 * F(pts)  # sum over three axes of the centre weight -5/2
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        lap += (4.0 / 3.0) * (F(pts + e) + F(pts - e)) - (1.0 / 12.0) * (F(pts + 2 * e) + F(pts - 2 * e))
    return lap / (h * h)


@pytest.mark.parametrize("N,alpha", [(4, 1.0), (8, 0.37), (12, 2.5)])
def test_fp_moments_are_the_fokker_planck_operator(N, alpha):
    """eq. scatter_moments: sigma_{s,n} - sigma_{s,0} = (alpha / 2) times the
    eigenvalue of the Laplace-Beltrami operator on degree n (Fokker-Planck
    equivalence); the eigenvalues come from finite differences."""
    fp = ang.fp_moments(alpha, N)
    assert fp.shape == (N + 1,)
    rng = np.random.default_rng(N)
    pts = rng.standard_normal((40, 3))
    pts /= np.linalg.norm(pts, axis=1)[:, None]
    Y = ang.real_harmonics(N, pts)
    lap = _laplace_beltrami_fd(N, pts)
    for n in range(N + 1):
        cols = slice(n * n, (n + 1) * (n + 1))
        pred = (fp[n] - fp[0]) * Y[:, cols]
        assert np.abs(alpha / 2 * lap[:, cols] - pred).max() < 2e-5 * max(1.0, np.abs(pred).max())
    # the expansion is truncated where the moments reach zero, and the
    # momentum-transfer (transport) cross section sigma_0 - sigma_1 is alpha
    assert abs(fp[N]) < 1e-12
    assert (np.diff(fp) < 0).all()


# ------------------------------------------------------------ particle balance

def _balance_terms(lv, phi, q_cell):
    g = lv.grid
    x = phi.reshape(lv.A, g.C, g.ns)
    ipsi = lv.basis_integral()                      # int psi_a (angular rule)
    cell_int = np.einsum('a,acl,l->c', ipsi, x, g.basis_int)   # int_{V_j} int_4pi phi
    removal = float(lv.sigma_t @ cell_int)
    scatter_in = float((lv.sigma_s * lv.moments[0]) @ cell_int)
    leak = 0.0
    for xi in range(g.dim):
        for side in (0, 1):
            nrm = 1.0 if side == 1 else -1.0
            cells = np.nonzero(g.coords[:, xi] == (g.n[xi] - 1 if side == 1 else 0))[0]
            fi = g.face_int[xi][side]
            for q in range(lv.P):
                if lv.signs[q][xi] * nrm <= 0:
                    continue  # incoming through this face: no outflow
                sel = lv.rule.owner == q
                om_psi = lv.rule.psi[q].T @ (lv.rule.w[sel] * lv.rule.omega[sel, xi])  # int Omega_xi psi_m
                for m in range(3):
                    leak += nrm * om_psi[m] * float(np.einsum('cl,l->', x[3 * q + m][cells], fi))
    source = 4.0 * math.pi * float(np.sum(q_cell)) * float(np.prod(g.h))
    return leak, removal, scatter_in, source


@pytest.mark.parametrize("dim,n,level,order,beam", [(3, 3, 1, 4, True), (2, 5, 2, 8, True), (3, 4, 1, 6, False)])
def test_particle_balance_of_a_converged_solve(dim, n, level, order, beam):
    prob = inputs.small_problem(dim=dim, n=n, level=level, order=order, g=0.85, c=0.95, seed=7, inflow=False)
    if beam:
        lo = (0, 1, 1 if dim == 3 else 0)
        hi = (0, n - 2, n - 2 if dim == 3 else 0)
        from dataclasses import replace
        prob = replace(prob, inflow=inputs.Inflow("beam", 0, 0, lo, hi, 1.3, (1.0, 0.0, 0.0)))
    op = OracleProblem(prob)
    b = op.rhs()
    sol = krylov.gmres(op.outer.apply_A, op.mg.vcycle, b, 1e-13, prob.restart)
    assert sol.converged
    leak, removal, scatter_in, source = _balance_terms(op.outer, sol.x, prob.q_cell)
    inflow = 0.0
    if beam:
        g = op.grid
        area = 1.0
        for a in range(1, dim):
            area *= (hi[a] - lo[a] + 1) * g.h[a]
        inflow = 1.3 * area
    lhs = leak + removal - scatter_in
    scale = leak + removal + scatter_in
    assert abs(lhs - (source + inflow)) < 1e-10 * scale
    # every term is non-trivial (a dropped term would not balance)
    assert leak > 1e-3 * scale and scatter_in > 1e-3 * scale


@pytest.mark.parametrize("N", [4, 16])
def test_paper_box_moments_follow_fp_moments(N):
    """The cube workloads' cross sections and moment ratios are eq.
    scatter_moments with transport cross section 1: sigma_s f_n equals the
    oracle's fp_moments(1, N) (pinned above), sigma_t = sigma_{s,0}, and the
    ratios beyond N vanish."""
    from paper_2010_04559_amd import inputs
    p = inputs.paper_box(N, level=1, n=3)
    fp = ang.fp_moments(1.0, N)
    m = p.moments(N + 3)
    assert np.allclose(p.sigma_s[0] * m[:N + 1], fp, rtol=0, atol=1e-12 * fp[0])
    assert not m[N + 1:].any()
    assert np.all(p.sigma_t == fp[0]) and np.all(p.sigma_s == fp[0])
    assert abs(p.sigma_s[0] * (m[0] - m[1]) - 1.0) < 1e-12
